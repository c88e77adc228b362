// Host planning of the hybrid reconstruction: range grid, reference
// wavenumbers, NUFFT parameters, back-projection tiling, workspace layout.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace pl {
namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) p0 = 1.0, p1 = z;
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Distance from a point to the axis-aligned rectangle [x0,x1] x [y0,y1].
double dist_to_rect(double px, double py, double x0, double x1, double y0, double y1) {
    const double cx = std::min(std::max(px, x0), x1), cy = std::min(std::max(py, y0), y1);
    return std::hypot(px - cx, py - cy);
}

}  // namespace

int make_plan(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts,
              HybridPlan* out) {
    if (!g || !grid || !out) return fail(PL_EINVAL, "null geometry, grid or plan");
    if (grid->nx < 1 || grid->ny < 1 || !(grid->dx > 0) || !(grid->dy > 0) ||
        !std::isfinite(grid->x0) || !std::isfinite(grid->y0))
        return fail(PL_EINVAL, "image grid needs nx, ny >= 1 and dx, dy > 0");
    if (static_cast<long long>(grid->nx) * grid->ny > (1LL << 26))
        return fail(PL_EUNSUPPORTED, "image grid has more than 2^26 pixels");
    HybridPlan p;
    p.mode = g->mode;
    p.n_ch = g->n_ch;
    p.n_z = g->n_scan;
    p.n_f = g->n_freq;
    p.scan_step = g->scan_step;
    p.nx = grid->nx;
    p.ny = grid->ny;
    p.x0 = grid->x0;
    p.y0 = grid->y0;
    p.dx = grid->dx;
    p.dy = grid->dy;
    if (opts) {
        p.precision = opts->precision;
        p.interp = opts->interp;
        if (opts->l_oversample != 0) p.sigma_l = opts->l_oversample;
        if (opts->nufft_tol != 0) p.tol = opts->nufft_tol;
        p.force_tile = opts->tile;
        p.force_kpl = opts->kz_per_lane;
        p.force_waves = opts->waves;
        p.force_bp_mfma = opts->mfma_backprojection;
        p.force_tile_y = opts->tile_y;
        p.force_kb = opts->kz_block;
        p.range_method = opts->range_method;
        p.ref_mode = opts->ref_mode;
    }
    if (p.ref_mode != PL_REF_BAND_CENTRE && p.ref_mode != PL_REF_MIN_K)
        return fail(PL_EINVAL, "unknown ref_mode %d", p.ref_mode);
    if (p.ref_mode == PL_REF_MIN_K) {
        // the paper's reference differs per k_z bin: its carrier is formed per
        // term, which only the k_z-per-lane back-projection does
        if (p.range_method != PL_RANGE_NUFFT)
            return fail(PL_EUNSUPPORTED, "ref_mode PL_REF_MIN_K takes the NUFFT range compression");
        if (p.force_bp_mfma > 0)
            return fail(PL_EUNSUPPORTED, "ref_mode PL_REF_MIN_K takes the VALU back-projection");
        if (p.force_kpl > 1 || p.force_kb != 0 || (p.force_waves != 0 && p.force_waves != 4))
            return fail(PL_EUNSUPPORTED, "ref_mode PL_REF_MIN_K runs one k_z bin per lane, 4 wavefronts");
    }
    if (p.force_kpl != 0 && p.force_kpl != 1 && p.force_kpl != 2 && p.force_kpl != 4)
        return fail(PL_EINVAL, "kz_per_lane must be 0, 1, 2 or 4");
    if (p.force_waves != 0 && p.force_waves != 4 && p.force_waves != 8)
        return fail(PL_EINVAL, "waves must be 0, 4 or 8");
    if (p.force_tile != 0 && p.force_tile != 16 && p.force_tile != 8 && p.force_tile != 4 && p.force_tile != 2)
        return fail(PL_EINVAL, "tile must be 0, 16, 8, 4 or 2");
    if (p.force_tile_y != 0 && p.force_tile_y != 16 && p.force_tile_y != 8)
        return fail(PL_EINVAL, "tile_y must be 0, 16 or 8");
    if (p.force_kb != 0 && p.force_kb != 32 && p.force_kb != 64 && p.force_kb != 128)
        return fail(PL_EINVAL, "kz_block must be 0, 32, 64 or 128");
    if (p.precision < PL_PREC_FP32 || p.precision > PL_PREC_FP16)
        return fail(PL_EINVAL, "unknown precision %d", p.precision);
    if (p.range_method != PL_RANGE_NUFFT && p.range_method != PL_RANGE_RESAMPLE)
        return fail(PL_EINVAL, "unknown range_method %d", p.range_method);
    if (p.range_method == PL_RANGE_RESAMPLE) {
        if (p.precision != PL_PREC_FP32)
            return fail(PL_EUNSUPPORTED, "the resampling range compression runs in FP32 only");
        if (p.n_f < 2) return fail(PL_EUNSUPPORTED, "the resampling range compression needs two frequencies");
    }
    if (p.interp < PL_INTERP_BSPLINE4 || p.interp > PL_INTERP_LINEAR)
        return fail(PL_EINVAL, "unknown interpolation %d", p.interp);
    if (!(p.sigma_l >= 2.0 && p.sigma_l <= 64.0)) return fail(PL_EINVAL, "l_oversample must be in [2, 64]");
    if (!(p.tol >= 1e-12 && p.tol <= 1e-2)) return fail(PL_EINVAL, "nufft_tol must be in [1e-12, 1e-2]");
    if (int rc = plan_axis_fft(p.n_z, &p.zfft)) return rc;

    // Dispersion k_rho = sqrt(k^2 - k_z^2 / 4) for the range l = rho_T + rho_R
    // (eq. 18; the monostatic eq. 5 is the same relation with l = 2 rho).
    // One reference wavenumber per block of k_z bins: the centre of the band
    // of k_rho it spans.  The reference cancels exactly between eqs. (8a) and
    // (8b); only the bandwidth of the range profiles depends on it.
    // Reference wavenumber of every k_z block and the range-grid step for a
    // given block size.
    auto set_blocks = [&](int block, double sigma) {
        p.block = std::max(block, kMinBlock);
        p.n_blocks = (p.n_z + p.block - 1) / p.block;  // <= kMaxScan / kMinBlock = kMaxBlocks
        double half_band = 0.0;
        for (int b = 0; b < p.n_blocks; ++b) {
            double lo = 1e300, hi = -1e300;
            for (int kap = b * p.block; kap < std::min(p.n_z, (b + 1) * p.block); ++kap) {
                const int sk = kap < (p.n_z + 1) / 2 ? kap : kap - p.n_z;
                const double kz = 2.0 * kPi * sk / (p.n_z * g->scan_step);
                for (int f = 0; f < p.n_f; ++f) {
                    const double arg = g->k[f] * g->k[f] - 0.25 * kz * kz;
                    if (arg <= 0) continue;
                    const double kr = std::sqrt(arg);
                    lo = std::min(lo, kr);
                    hi = std::max(hi, kr);
                }
            }
            if (hi < lo) {
                p.kref[b] = 0.0;
            } else {
                p.kref[b] = 0.5 * (lo + hi);
                half_band = std::max(half_band, 0.5 * (hi - lo));
            }
        }
        if (p.ref_mode == PL_REF_MIN_K) {
            // the paper's k_rho0 = k_rho at the lowest wavenumber k_0 (the
            // smallest real k_rho of the bin where k_0 is evanescent): k' runs
            // over [0, max k_rho - k_rho0], so the range grid resolves the
            // widest such band
            half_band = 0.0;
            for (int kap = 0; kap < p.n_z; ++kap) {
                const int sk = kap < (p.n_z + 1) / 2 ? kap : kap - p.n_z;
                const double kz = 2.0 * kPi * sk / (p.n_z * g->scan_step);
                double lo = -1.0, hi = -1.0;
                for (int f = 0; f < p.n_f; ++f) {
                    const double arg = g->k[f] * g->k[f] - 0.25 * kz * kz;
                    if (arg <= 0) continue;
                    const double kr = std::sqrt(arg);
                    if (lo < 0) lo = kr;
                    hi = kr;
                }
                if (lo >= 0) half_band = std::max(half_band, hi - lo);
            }
        }
        if (half_band <= 0) half_band = 1.0;  // single frequency, no k_z spread
        p.half_band = half_band;
        p.sigma_used = sigma;
        p.du = kPi / (sigma * half_band);
    };

    // MFMA back-projection (BF16 / FP16 modes): tiles of 4x4 pixel groups,
    // each group's taps inside one 16-sample window that starts on a multiple
    // of 4 samples.  |l(p) - l(q)| <= 2 |p - q|, so a group's first tap is at
    // most 3 samples past its window start and its last at most
    // ceil(2 * diagonal / du) + 3 past its first.  The kernel forms each
    // pixel's position in float32 from its tile centre's (error far below
    // 1e-3 samples), so the plan keeps 2 * diagonal / du <= 8.99: a floor
    // taken in float32 then never spreads a group's first taps over more
    // than 9 samples.
    p.bp_mfma = false;
    p.bp_mfma_sp = false;
    if (p.force_bp_mfma > 2) return fail(PL_EINVAL, "mfma_backprojection must be -1, 0, 1 or 2");
    if (p.force_bp_mfma > 0) {
        if (p.precision == PL_PREC_FP32)
            return fail(PL_EUNSUPPORTED, "the MFMA back-projection runs in the BF16 / FP16 modes only");
        // single pass: one FP16 product per pair (scaled FP16 profiles)
        const bool sp = p.force_bp_mfma == 2;
        if (sp && p.precision != PL_PREC_FP16)
            return fail(PL_EUNSUPPORTED, "the single-pass MFMA back-projection runs in the FP16 mode only");
        if (p.force_kpl != 0)
            return fail(PL_EINVAL, "kz_per_lane applies to the VALU back-projection");
        const int tx = p.force_tile ? p.force_tile : 16;
        const int ty = p.force_tile_y ? p.force_tile_y : tx;
        if (!((tx == 8 && ty == 8) || (tx == 16 && (ty == 8 || ty == 16))))
            return fail(PL_EINVAL, "MFMA back-projection tiles are 8x8, 16x8 or 16x16");
        const int kb = p.force_kb ? p.force_kb : 64;
        if (kb == 32) return fail(PL_EINVAL, "the MFMA back-projection takes 64 or 128 k_z bins per workgroup");
        // eight wavefronts (two 4x4 groups each) on the 16x16 and 16x8 tiles
        // with 64 k_z bins: measured fastest on gfx950
        const double gdiag = std::hypot(3.0 * grid->dx, 3.0 * grid->dy);
        set_blocks(kb, p.sigma_l);
        if (2.0 * gdiag / p.du > 8.99) {
            // widest grid step that fits, as long as the oversampling stays >= 4
            const double du_fit = 2.0 * gdiag / 8.99;
            const double sigma_fit = kPi / (du_fit * p.half_band);
            if (sigma_fit >= 4.0) set_blocks(kb, std::min(p.sigma_l, sigma_fit));
        }
        // staged window: every tap of the tile plus alignment (8-sample
        // chunks), and one sample against float rounding
        const double rt = 0.5 * std::hypot((tx - 1) * grid->dx, (ty - 1) * grid->dy);
        const int need = static_cast<int>(std::ceil(4.0 * rt / p.du)) + 7;
        const int nck = std::max(2, (need + 7) / 8);
        const size_t lds = backproject_mfma_lds_bytes(kb, sp);
        if (2.0 * gdiag / p.du <= 8.995 && nck <= 8 && lds <= kMaxLds && p.n_f <= 128) {
            p.bp_mfma = true;
            p.bp_mfma_sp = sp;
            p.tile_x = tx;
            p.tile_y = ty;
            p.window = 8 * nck;  // samples staged per plane and row
            p.window_pad = sp ? 17 : 33;  // LDS row length in 16-byte chunks (2 or 4 planes x 8 + 1)
            p.waves = p.force_waves ? p.force_waves : ((tx * ty >= 128 && kb == 64) ? 8 : 4);
            if (tx * ty == 64 && p.waves == 8)
                return fail(PL_EUNSUPPORTED, "8 wavefronts need a 16x8 or 16x16 MFMA tile");
            if (tx * ty == 256 && kb == 128 && p.waves == 8)
                return fail(PL_EUNSUPPORTED, "8 wavefronts with a 16x16 tile take 64 k_z bins");
        }
    }
    if (p.force_bp_mfma > 0 && !p.bp_mfma)
        return fail(PL_EUNSUPPORTED, "the MFMA back-projection does not fit this grid");
    // VALU back-projection: the pixel-per-lane kernel when its 8x8 tile's
    // window fits (32 k_z bins per workgroup by default: the narrower k'
    // band of a smaller block coarsens the range grid, and with 64 bins the
    // row buffers halve the workgroups per CU), else one k_z bin per lane
    // (one bin per lane by default:
    // more bins per lane make the staged window too large for several
    // resident workgroups per CU).
    p.bp_gather = false;
    if (!p.bp_mfma) {
        if (p.force_tile == 16 || p.force_tile_y != 0)
            return fail(PL_EINVAL, "tile 16 and tile_y apply to the MFMA back-projection");
        if (p.force_kb && (p.force_kb > 64 || p.force_kpl))
            return fail(PL_EINVAL, "the VALU back-projection takes kz_block 32 or 64 (pixel-per-lane kernel)");
        if (p.force_kpl == 0 && (p.force_tile == 0 || p.force_tile == 8) &&
            (p.force_waves == 0 || p.force_waves == 4) && p.ref_mode == PL_REF_BAND_CENTRE) {
            // staged rows start on an even sample (16-byte copies) and hold
            // the window: the taps of every pixel of the 8x8 tile and the
            // sample after them (a pixel reads three aligned chunks around
            // its four taps), ceil(2 reach / du) + 7 samples with reach = 2 rt,
            // and one more against float rounding
            set_blocks(p.force_kb ? p.force_kb : 32, p.sigma_l);
            const double rt = 0.5 * std::hypot(7.0 * grid->dx, 7.0 * grid->dy);
            const int nchk = (static_cast<int>(std::ceil(4.0 * rt / p.du)) + 8 + 1) / 2;  // 2-sample chunks
            const int rows[6] = {12, 14, 18, 24, 32, 40};   // compiled row classes
            int rsc = 0;
            for (int r : rows)
                if (!rsc && nchk <= r) rsc = r;
            if (rsc && backproject_gather_lds_bytes(p.block, rsc) <= kMaxLds) {
                p.bp_gather = true;
                p.tile_x = p.tile_y = 8;
                p.window = 2 * nchk;   // samples staged per row
                p.window_pad = rsc;    // LDS row length in 16-byte chunks
                p.waves = 4;
            }
        }
        if (!p.bp_gather) {
            if (p.force_kb) return fail(PL_EUNSUPPORTED, "kz_block needs the pixel-per-lane back-projection");
            set_blocks(kLanes * (p.force_kpl ? p.force_kpl : 1), p.sigma_l);
        }
    }

    // Range window of every channel over the pixel-centre rectangle.
    const double gx1 = grid->x0 + (grid->nx - 1) * grid->dx, gy1 = grid->y0 + (grid->ny - 1) * grid->dy;
    double span = 0.0;
    for (int c = 0; c < p.n_ch; ++c) {
        const double tx = g->tx[2 * c], ty = g->tx[2 * c + 1], rx = g->rx[2 * c], ry = g->rx[2 * c + 1];
        const double lmin = dist_to_rect(tx, ty, grid->x0, gx1, grid->y0, gy1) +
                            dist_to_rect(rx, ry, grid->x0, gx1, grid->y0, gy1);
        double lmax = 0.0;
        for (int i = 0; i < 4; ++i) {
            const double x = (i & 1) ? gx1 : grid->x0, y = (i & 2) ? gy1 : grid->y0;
            lmax = std::max(lmax, std::hypot(x - tx, y - ty) + std::hypot(x - rx, y - ry));
        }
        span = std::max(span, lmax - lmin);
    }

    // k_z-per-lane kernel tile: the staged range window must hold every tap
    // of the tile's pixels (|l(p) - l(centre)| <= 2 * half-diagonal).  Prefer
    // the largest tile whose window fits 64 samples (one staging load per
    // lane and row; the 2x2 fallback allows 128) and whose LDS (window starts
    // + two staged windows of 64 x kz_per_lane rows) fits the workgroup's
    // 160 KiB.
    if (!p.bp_mfma && !p.bp_gather) {
        const int tiles[3][2] = {{8, 8}, {4, 4}, {2, 2}};
        p.window = 0;
        for (int t = 0; t < 3; ++t) {
            if (p.force_tile && tiles[t][0] != p.force_tile) continue;
            const double rt = 0.5 * std::hypot((tiles[t][0] - 1) * grid->dx, (tiles[t][1] - 1) * grid->dy);
            const int wl = static_cast<int>(std::ceil(4.0 * rt / p.du)) + 6;
            const size_t lds = backproject_lds_bytes(p.n_ch, p.block, wl | 1);
            if ((wl <= (t == 2 ? 128 : 64) && lds <= kMaxLds) || t == 2 || p.force_tile) {
                p.tile_x = tiles[t][0];
                p.tile_y = tiles[t][1];
                p.window = wl;
                break;
            }
        }
        p.waves = p.force_waves ? p.force_waves : 4;
        if (p.waves == 8 && p.tile_x != 8)
            return fail(PL_EUNSUPPORTED, "8 wavefronts per workgroup need the 8x8 tile");
        if (backproject_lds_bytes(p.n_ch, p.block, p.window | 1) > kMaxLds)
            return fail(PL_EUNSUPPORTED, "back-projection staging exceeds the LDS (lower kz_per_lane)");
        p.window_pad = p.window | 1;  // odd row length: conflict-free LDS reads across lanes
    }
    if (p.window > 128)
        return fail(PL_EUNSUPPORTED, "pixels are too coarse for the range grid (window %d > 128)", p.window);
    p.tiles_x = (grid->nx + p.tile_x - 1) / p.tile_x;
    p.tiles_y = (grid->ny + p.tile_y - 1) / p.tile_y;

    // range samples: a multiple of 4 (8-byte stores of split BF16 profiles).
    // The NUFFT's fine grid: for FP32 NUFFT plans the smallest grid of at
    // least 1.25 n_l points, preferring the 64 R sizes (R 2,3,5-smooth, at
    // most 32) of the wavefront-per-pair kernels; other plans keep 2 n_l
    // (2,3,5-smooth; the resampling method's uniform grid and the plan
    // tables use it).
    int nl = static_cast<int>(std::ceil(span / p.du)) + 8;
    nl = std::max(nl, p.window + 2);
    nl = (nl + 3) & ~3;
    const bool nufft32 = p.precision == PL_PREC_FP32 && p.range_method == PL_RANGE_NUFFT;
    if (nufft32) {
        const int want = static_cast<int>(std::ceil(kNufftUpsample * nl));
        int nf = 0;
        for (int r = (want + 63) / 64; r <= 32 && !nf; ++r)
            if (is_fft_friendly(r)) nf = 64 * r;
        if (!nf)
            for (nf = want; !is_fft_friendly(nf); ++nf) {
            }
        p.n_l = nl;
        p.n_fine = nf;
    } else {
        while (!is_fft_friendly(2 * nl)) nl += 4;
        p.n_l = nl;
        p.n_fine = 2 * nl;
    }
    if (p.n_fine > kMaxFine)
        return fail(PL_EUNSUPPORTED, "range grid of %d samples needs a fine grid over %d (lower l_oversample)", p.n_l,
                    kMaxFine);
    factor_radices(p.n_fine, &p.fine_rad);
    if (p.range_method == PL_RANGE_RESAMPLE) {
        // uniform k_L grid whose inverse FFT lands on the range grid: step
        // 2 pi / (n_fine du); a block's band of 2 half_band holds at most
        // n_fine / sigma + 1 of its points, so they never share a bin
        p.dkl = 2.0 * kPi / (p.n_fine * p.du);
        p.k0 = g->k[0];
        p.dk = (g->k[p.n_f - 1] - g->k[0]) / (p.n_f - 1);
        if (!(p.dk > 0) || 2.0 * p.half_band / p.dkl + 2.0 > p.n_fine)
            return fail(PL_EUNSUPPORTED, "resampling grid does not fit the range grid");
        // reference wavenumbers on the grid (the reference cancels between
        // eqs. 8a and 8b, any value is exact): the grid's k' are then whole
        // multiples of dkl and land on FFT bins without a residual shift.  The
        // band edges move by at most dkl / 2 = sigma half_band / n_fine.
        for (int b = 0; b < p.n_blocks; ++b) p.kref[b] = p.dkl * std::nearbyint(p.kref[b] / p.dkl);
    }

    // Exponential-of-semicircle kernel exp(beta (sqrt(1 - z^2) - 1)) of
    // width W (Barnett, Magland, af Klinteberg 2019).  For the 2x fine grid:
    // W = ceil(log10(1/tol)) + 1, beta = 2.30 W.  For an upsampling factor
    // s = n_fine / n_l below 2, their error estimate exp(-pi W sqrt(1 - 1/s))
    // gives W = ceil(ln(1/tol) / (pi sqrt(1 - 1/s))), and beta =
    // 0.97 pi W (1 - 1/(2 s)).
    const double ups = static_cast<double>(p.n_fine) / p.n_l;
    if (ups >= 1.999) {
        p.W = std::max(2, static_cast<int>(std::ceil(std::log10(1.0 / p.tol))) + 1);
        p.W = std::min(p.W, 16);
        p.beta = 2.30 * p.W;
    } else {
        p.W = std::max(2, static_cast<int>(std::ceil(std::log(1.0 / p.tol) / (kPi * std::sqrt(1.0 - 1.0 / ups)))));
        p.W = std::min(p.W, 16);
        p.beta = 0.97 * kPi * p.W * (1.0 - 0.5 / ups);
    }
    p.h = 0.5 * p.W;
    if (p.n_fine / p.sigma_l + 2 * p.W + 2 >= p.n_fine) return fail(PL_EUNSUPPORTED, "fine grid too short");
    p.n_gl = std::min(kMaxGL, 4 * p.W + 16);
    gauss_legendre(p.n_gl, p.gl_x, p.gl_w);

    // interpolation weights as cubic polynomials in t = u - floor(u), taps at
    // floor(u) - 1 .. floor(u) + 2
    static const float bsp[4][4] = {{1.f / 6, -0.5f, 0.5f, -1.f / 6},
                                    {4.f / 6, 0.f, -1.f, 0.5f},
                                    {1.f / 6, 0.5f, 0.5f, -0.5f},
                                    {0.f, 0.f, 0.f, 1.f / 6}};
    static const float lag[4][4] = {{0.f, -1.f / 3, 0.5f, -1.f / 6},
                                    {1.f, -0.5f, -1.f, 0.5f},
                                    {0.f, 1.f, 0.5f, -0.5f},
                                    {0.f, -1.f / 6, 0.f, 1.f / 6}};
    static const float lin[4][4] = {{0.f, 0.f, 0.f, 0.f}, {1.f, -1.f, 0.f, 0.f}, {0.f, 1.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    const float(*src)[4] = p.interp == PL_INTERP_BSPLINE4 ? bsp : (p.interp == PL_INTERP_LAGRANGE4 ? lag : lin);
    std::memcpy(p.coef, src, sizeof(p.coef));

    // workspace layout
    const size_t nch = p.n_ch, nz = p.n_z, nf = p.n_f, npix = static_cast<size_t>(p.nx) * p.ny;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    p.off_spec = take(nch * nz * nf * 8);
    p.off_q = take(nch * nz * static_cast<size_t>(p.n_l) * 8);
    p.off_G = take(npix * nz * 8);
    p.off_llo = take(nch * 8);
    p.off_lref = take(nch * 8);
    p.off_zfft = take(p.zfft.bytes);
    p.off_tw_fine = take(static_cast<size_t>(p.n_fine) * 8);
    p.off_deap = take(static_cast<size_t>(p.n_l) * 4);
    p.off_kp = take(nz * nf * 8);
    p.off_wk = take(nz * nf * 4);
    p.off_krz = take(nz * 8);
    p.off_tiles = take(tile_table_bytes(p));
    p.off_part = take(backproject_mfma_part_bytes(p));
    p.n_chp = (p.n_ch + 31) / 32 * 32;
    p.n_fp = (p.n_f + 15) / 16 * 16;
    if (p.precision != PL_PREC_FP32) {
        if (p.n_fp > 128)
            return fail(PL_EUNSUPPORTED, "MFMA range compression supports up to 128 frequencies");
        p.off_mfma_a = take(nz * static_cast<size_t>(p.n_chp) * 4);
        p.off_qexp = take(4 * (kProfileScaleParts + 1));
        p.off_mfma_b = take(nz * static_cast<size_t>(p.n_chp) * 4 * p.n_fp * 2);
    } else {
        p.off_mfma_a = off;
        p.off_mfma_b = off;
        p.off_qexp = off;
    }
    p.total = off;
    *out = p;
    return PL_OK;
}

}  // namespace pl
