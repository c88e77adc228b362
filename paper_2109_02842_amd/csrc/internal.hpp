// Internal declarations of the polyrecon library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/polyrecon.h"

namespace pl {

constexpr double kSpeedOfLight = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr int kLanes = 64;          // wavefront width on gfx950
constexpr int kMaxScan = 4096;
constexpr int kMinBlock = 32;       // fewest k_z bins sharing one reference wavenumber
constexpr int kMaxBlocks = kMaxScan / kMinBlock;
constexpr int kMaxChirpLen = 8192;  // longest smooth length a chirp-z transform runs through
// single-pass FP16 profiles: workgroups of the exponent reduction; the
// workspace slot holds their parts, then the scale exponent g
constexpr int kProfileScaleParts = 64;
constexpr size_t kMaxLds = 160 * 1024;          // LDS per workgroup on gfx950
constexpr int kMaxFreq = 1024;
constexpr int kMaxFine = 4096;      // NUFFT fine grid held twice in LDS (64 KiB)
constexpr double kNufftUpsample = 1.25;  // FP32 NUFFT: fine grid of at least 1.25 n_l points
constexpr int kMaxGL = 64;          // quadrature nodes for the kernel transform
constexpr int kMaxRadices = 16;

// ---------------------------------------------------------------- errors
int fail(int code, const char* fmt, ...);
void clear_error();
int check_launch(const char* what);

// ------------------------------------------------------- device geometry
struct DeviceTables {
    double* chan = nullptr;  // [n_ch][4]: x_T, y_T, x_R, y_R
    double* k = nullptr;     // [n_freq] wavenumbers
};

// Radix plan of a transform length (radices in {8, 4, 2, 3, 5}).
struct Radices {
    int n = 0;
    int count = 0;
    int r[kMaxRadices] = {};
};
bool factor_radices(int n, Radices* out);
bool is_fft_friendly(int n);

// A batched transform of length n along a strided axis (the scan FFT of
// eq. 2/12 and the k_z inverse FFT of eq. 9).  A 2,3,5-smooth n runs as
// mixed-radix stages of length m = n; any other n by Bluestein's chirp-z
// transform through the smallest smooth m >= 2 n - 1.  Its tables live in a
// caller's buffer at byte offsets from a table base: m twiddles
// exp(-2 pi i t / m); for the chirp-z form also the chirp exp(-i pi t^2 / n)
// (n values), the padded conjugate chirp (m values, scratch of the table
// step) and its forward transform scaled by 1/m (m values).
struct AxisFft {
    int n = 0, m = 0;
    bool chirp = false;
    Radices rad;  // radices of m
    size_t off_tw = 0, off_chirp = 0, off_pad = 0, off_hat = 0, bytes = 0;
};
int plan_axis_fft(int n, AxisFft* out);
// Writes the tables of f at `tables` (256-byte aligned, f.bytes long).
int launch_axis_fft_tables(const AxisFft& f, char* tables, hipStream_t s);

}  // namespace pl

struct pl_geometry {
    int mode = PL_MONO;
    int n_chords = 0, n_elem = 0, n_tx = 0, n_scan = 0, n_freq = 0, n_ch = 0;
    double radius = 0, arc_center = 0, spacing = 0, scan_step = 0, scan_z0 = 0;
    double f_start = 0, f_stop = 0;
    std::vector<double> tx_off;          // chord-local Tx offsets (multi)
    std::vector<double> tx, rx;          // [n_ch][2]
    std::vector<double> z, f, k;         // scan heights, frequencies, wavenumbers
    std::vector<double> ends;            // [n_chords][2][2]
    std::vector<double> chan;            // [n_ch][4]: x_T, y_T, x_R, y_R (source of the device copy)
    mutable std::mutex mu;
    mutable std::map<int, pl::DeviceTables> dev;

    // Device tables for the current device.  If there are none yet and
    // upload is true they are allocated and copied in stream order on
    // `stream` (the copies read chan and k, which live as long as the
    // handle); with upload false that is an error (PL_EINVAL).
    int device_tables(pl::DeviceTables* out, hipStream_t stream = nullptr, bool upload = true) const;
    ~pl_geometry();
};

namespace pl {

// Host-side plan of a hybrid reconstruction: every size and scalar the
// kernels need, and the workspace layout.
struct HybridPlan {
    int mode = 0, n_ch = 0, n_z = 0, n_f = 0;
    int n_chp = 0, n_fp = 0;  // channels padded to 32, frequencies to 16 (MFMA tiles)
    double scan_step = 0;
    int nx = 0, ny = 0;
    double x0 = 0, y0 = 0, dx = 0, dy = 0;
    int precision = PL_PREC_FP32, interp = PL_INTERP_BSPLINE4;
    double sigma_l = 6.0, tol = 1e-6;
    int force_tile = 0, force_tile_y = 0, force_kpl = 0, force_waves = 0, force_bp_mfma = 0, force_kb = 0;
    bool bp_mfma = false;            // back-projection on the matrix cores (split-BF16 q)
    bool bp_mfma_sp = false;         // its single-pass form (scaled FP16 q, one product per pair)
    bool bp_gather = false;          // VALU back-projection with one pixel per lane
    int range_method = PL_RANGE_NUFFT;
    int ref_mode = PL_REF_BAND_CENTRE;  // reference wavenumber: per k_z block, or the paper's per k_z
    double dkl = 0, k0 = 0, dk = 0;  // resampling: uniform k_L step, frequency grid start and step
    double half_band = 0, sigma_used = 0;
    // range grid and NUFFT
    int n_l = 0, n_fine = 0, W = 0;
    double du = 0, h = 0, beta = 0;
    int block = kLanes;  // k_z bins sharing one reference wavenumber (64 x bins per lane)
    int n_blocks = 0;
    double kref[kMaxBlocks] = {};
    AxisFft zfft;        // the scan and k_z transforms (length n_z)
    Radices fine_rad;
    int n_gl = 0;
    double gl_x[kMaxGL] = {}, gl_w[kMaxGL] = {};
    // back-projection tiling
    int tile_x = 8, tile_y = 8, tiles_x = 0, tiles_y = 0, window = 0, window_pad = 0, waves = 4;
    // interpolation weights w_k(t) = sum_j coef[k][j] t^j, taps at floor(u)-1+k
    float coef[4][4] = {};
    // workspace layout (byte offsets, 256-aligned)
    size_t off_spec = 0, off_q = 0, off_G = 0, off_llo = 0, off_lref = 0, off_zfft = 0, off_tw_fine = 0;
    size_t off_deap = 0, off_kp = 0, off_wk = 0, off_krz = 0, off_mfma_a = 0, off_mfma_b = 0, off_tiles = 0,
           off_qexp = 0, off_part = 0, total = 0;
};

// Per (pixel tile, channel) geometry, computed once per call in float64
// (tile-major: entry tile * n_ch + c).  A pixel's range follows from the
// tile centre's in float32 without loss: with X the vector from an antenna
// to the centre, D = |X| and d the pixel's offset from the centre,
// |X + d| - D = s / (D + sqrt(D^2 + s)), s = 2 X.d + d.d, a difference of at
// most a tile diagonal, exact to float32 rounding.
struct GatherTileEntry {
    double lc;             // range rho_T + rho_R from the channel to the tile centre
    int win;               // first staged sample of the tile's window (even)
    int base;              // floor(u(centre)) - 1 - win
    float uf;              // u(centre) - floor(u(centre)), u = (l - l_lo) / du
    float xt, yt, dt;      // centre minus Tx position, and its length
    float xr, yr, dr;      // centre minus Rx position, and its length
    float pad_;
};
static_assert(sizeof(GatherTileEntry) == 48, "tile table entry");
// After the n_tiles * n_ch entries the tile table holds the centres'
// carriers exp(j k_ref(b) l_c) for every k_z block b (float64 phase, range
// reduced, then float32): float2 at ((b * n_tiles + tile) * n_ch + c).

size_t backproject_lds_bytes(int n_ch, int rows, int window_pad);
size_t backproject_mfma_lds_bytes(int kz_block, bool single_pass);
// Partial spectra of the matrix-core back-projection's split tail items (at
// most kMaxTailPieces pieces of a tile x k_z block each; 0 for other plans).
constexpr int kMaxTailPieces = 1024;
size_t backproject_mfma_part_bytes(const HybridPlan& p);
size_t backproject_gather_lds_bytes(int rows, int row_chunks);

// Batched pixel-per-lane back-projection (one persistent launch for several
// scans): a per-scan descriptor of gather_batch_desc_bytes() bytes, built on
// the host; work items are int4 (scan, k_z block, tile, 0) in eight
// contiguous per-XCD queues delimited by bounds[0..8] (device ints); eight
// counters (unsigned) live in the caller's workspace.
size_t gather_batch_desc_bytes();
int build_gather_batch_desc(const HybridPlan& p, size_t ws_off, int rsc, void* out);
int gather_batch_grid(int kb, int rsc, size_t smem, int* blocks);
int launch_gather_batch(const void* descs, const void* items, const int* bounds, unsigned* counters, char* ws,
                        int kb, int rsc, size_t smem, int blocks, hipStream_t s);
int make_plan(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts,
              HybridPlan* p);

// The hybrid reconstruction (reconstruct_hybrid and its variants): tables =
// false skips the plan-table step (ws prepared by hybrid_prepare); upload =
// false takes the geometry's device tables as already uploaded (no
// allocation; PL_EINVAL if they are not); what names the entry point in
// error messages; ev: optional stage events.
int reconstruct_impl(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts, const float* echo,
                     float* image, void* ws, size_t ws_bytes, hipEvent_t* ev, hipStream_t stream, bool tables,
                     bool upload, const char* what);

// ---------------------------------------------------------- launchers
int launch_plan_tables(const HybridPlan& p, const DeviceTables& dt, char* ws, hipStream_t s);
// Per (tile, channel) geometry of the pixel-per-lane and matrix-core
// back-projections (after the plan tables: reads l_lo); a no-op for plans
// without those kernels.
size_t tile_table_bytes(const HybridPlan& p);
int launch_tile_tables(const HybridPlan& p, const DeviceTables& dt, char* ws, hipStream_t s);
// The transforms take the tables of f at `tables`.
int launch_scan_fft(const pl_geometry* g, const float2* echo, float2* spec, const AxisFft& f, const char* tables,
                    hipStream_t s);
int launch_range_compress_fp32(const HybridPlan& p, const float2* spec, char* ws, float2* q,
                               hipStream_t s);
int launch_range_compress_resample(const HybridPlan& p, const float2* spec, char* ws, float2* q,
                                   hipStream_t s);
int launch_range_compress_mfma(const HybridPlan& p, const float2* spec, char* ws, float2* q,
                               hipStream_t s);
int launch_range_compress_mfma_split(const HybridPlan& p, const float2* spec, char* ws,
                                     unsigned short* qs, hipStream_t s);
int launch_backproject(const HybridPlan& p, const DeviceTables& dt, const float2* q, char* ws,
                       float2* G, hipStream_t s);
int launch_backproject_mfma(const HybridPlan& p, const DeviceTables& dt, const unsigned short* qs,
                            char* ws, float2* G, hipStream_t s);
int launch_kz_ifft(const HybridPlan& p, const float2* G, float2* image, const char* tables, hipStream_t s);
// Adjoint steps (image -> echo), in the order they run.
int launch_kz_fft_adjoint(const HybridPlan& p, const float2* image, float2* Gt, const char* tables, hipStream_t s);
int launch_backproject_adjoint(const HybridPlan& p, const DeviceTables& dt, const float2* Gt, char* ws, float2* qt,
                               hipStream_t s);
int launch_range_adjoint(const HybridPlan& p, const float2* qt, char* ws, float2* St, hipStream_t s);
int launch_scan_fft_adjoint(const pl_geometry* g, const float2* St, float2* echo, const AxisFft& f,
                            const char* tables, hipStream_t s);
int launch_simulate(const pl_geometry* g, const DeviceTables& dt, int n_scat, const double* xyz,
                    const double* refl, float2* echo, hipStream_t s);
// Brute-force BP over image planes [iz0, iz0 + nz): workspace layout (the
// k_f-weighted echo, then, when the (channel, scan) rows are split over
// n_seg workgroup segments, their partial images [n_seg][nz][ny][nx]).
struct BpLayout {
    int ch = 1, n_seg = 1;          // rows staged per LDS buffer; row segments
    long long rows_per_seg = 0;
    size_t off_part = 0, bytes = 0;
};
BpLayout bp_layout(const pl_geometry* g, const pl_image_grid* grid, int nz);
int launch_bp(const pl_geometry* g, const DeviceTables& dt, const pl_image_grid* grid, int iz0,
              int nz, const float2* echo, char* ws, float2* image, hipStream_t s);

}  // namespace pl
