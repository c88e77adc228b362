// Point-scatterer echo simulation, eq. (1) (monostatic) and eq. (10)
// (multistatic), and brute-force back-projection (the paper's comparison
// method).
#include "device.hpp"

namespace pl {
namespace {

constexpr int kSimChunk = 16;  // frequencies per thread

struct SimArgs {
    int n_ch, n_z, n_f, n_scat, n_chunks, pad_;
    double z0, dz, dk;
};

// One thread per (channel, scan position, chunk of 16 frequencies).  For
// every scatterer the two-way path D = R_T + R_R is formed in float64; the
// phasor exp(-j k_f D) is evaluated directly (float64 range reduction) at the
// chunk's first frequency and advanced by exp(-j dk D) within the chunk.
__global__ __launch_bounds__(256) void simulate_kernel(const double* __restrict__ chan,
                                                       const double* __restrict__ k,
                                                       const double* __restrict__ xyz,
                                                       const double* __restrict__ refl, SimArgs a,
                                                       float2* __restrict__ echo) {
    const long long t = blockIdx.x * 256LL + threadIdx.x;
    const long long total = static_cast<long long>(a.n_ch) * a.n_z * a.n_chunks;
    if (t >= total) return;
    const int chunk = static_cast<int>(t % a.n_chunks);
    const long long cm = t / a.n_chunks;
    const int m = static_cast<int>(cm % a.n_z);
    const int c = static_cast<int>(cm / a.n_z);
    const int f0 = chunk * kSimChunk;
    const int nfc = min(kSimChunk, a.n_f - f0);
    const double xt = chan[4 * c], yt = chan[4 * c + 1], xr = chan[4 * c + 2], yr = chan[4 * c + 3];
    const double zm = a.z0 + m * a.dz;
    const double k0_rev = k[f0] * (0.5 / kPi), dk_rev = a.dk * (0.5 / kPi);
    float2 acc[kSimChunk];
#pragma unroll
    for (int f = 0; f < kSimChunk; ++f) acc[f] = make_float2(0.f, 0.f);
    for (int s = 0; s < a.n_scat; ++s) {
        const double px = xyz[3 * s], py = xyz[3 * s + 1], pz = xyz[3 * s + 2];
        const float2 sig = make_float2(static_cast<float>(refl[2 * s]), static_cast<float>(refl[2 * s + 1]));
        const double dzp = pz - zm;
        const double d = sqrt((px - xt) * (px - xt) + (py - yt) * (py - yt) + dzp * dzp) +
                         sqrt((px - xr) * (px - xr) + (py - yr) * (py - yr) + dzp * dzp);
        float2 v = cmul(sig, cis_rev(-k0_rev * d));
        const float2 st = cis_rev(-dk_rev * d);
#pragma unroll
        for (int f = 0; f < kSimChunk; ++f) {
            acc[f] = cadd(acc[f], v);
            v = cmul(v, st);
        }
    }
    float2* out = echo + (static_cast<size_t>(c) * a.n_z + m) * a.n_f + f0;
#pragma unroll
    for (int f = 0; f < kSimChunk; ++f)
        if (f < nfc) out[f] = acc[f];
}

__global__ void weight_echo_kernel(const float2* __restrict__ echo, const double* __restrict__ k, int n_f,
                                   long long total, float2* __restrict__ out) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= total) return;
    out[i] = cscale(echo[i], static_cast<float>(k[i % n_f]));
}

// sqrt(x) for x >= 0 to double precision: hardware FP32 root (about 1 ulp),
// then one Newton step whose residual is formed in FP64.
__device__ __forceinline__ double sqrt_dp(double x) {
    const float r = __builtin_amdgcn_sqrtf(static_cast<float>(x));
    const double rd = r;
    const float corr = static_cast<float>(x - rd * rd) * (0.5f * __builtin_amdgcn_rcpf(r));
    return r > 0.f ? rd + static_cast<double>(corr) : 0.0;
}

struct BpArgs {
    int n_ch, n_z, n_f, nx, ny, tiles_x, n_tiles, n_groups, iz_first, iz_out0, nz_out, rows_per_seg, ch, mono;
    long long n_rows;
    double x0, y0, dx, dy, dz, k0_rev, dk_rev;
};

constexpr int kBpTile = 16;       // pixels per tile edge: 256 lanes, one pixel each
constexpr int kBpStageElems = 4096;  // complex echo samples staged per buffer (32 KiB)
constexpr int kBpFreqBlock = 32;  // frequencies per Horner block

// Brute-force back-projection.  Workgroup = 16 x 16 pixels (lane = pixel) x
// VPL image planes (every lane sums VPL voxels) x one segment of the
// (channel, scan position) rows.  The segment's k_f-weighted echo rows are
// staged in LDS, ch rows at a time, double-buffered (the next stage's loads
// are in flight while the current one is summed), and every wavefront reads
// them by broadcast.  Per (voxel, row): the path D = R_T + R_R in float64,
// z = exp(j dk D) from a float64-reduced phase, and the frequency sum
// sum_f a_f exp(j k_f D) = sum_blocks exp(j k_b D) sum_f' a_(b+f') z^f' with
// the inner sums by Horner's rule (one complex multiply-add, four FMAs, per
// frequency) over blocks of 32 frequencies, each anchored by its own
// float64-reduced phase exp(j k_b D).  The segment's sums go to out (the
// image, or the segment's plane of partial sums) in a fixed order.
template <int VPL>
__global__ __launch_bounds__(256) void bp_tile_kernel(const float2* __restrict__ sw, const double* __restrict__ chan,
                                                      BpArgs a, float2* __restrict__ out) {
    constexpr int PRE = kBpStageElems / 256;
    extern __shared__ float2 rows[];   // [2][ch * n_f]
    const int tile = blockIdx.x % a.n_tiles;
    const int rest = blockIdx.x / a.n_tiles;
    const int grp = rest % a.n_groups, seg = rest / a.n_groups;
    const int tid = threadIdx.x;
    const int px = (tile % a.tiles_x) * kBpTile + (tid & (kBpTile - 1));
    const int py = (tile / a.tiles_x) * kBpTile + tid / kBpTile;
    const double x = a.x0 + px * a.dx, y = a.y0 + py * a.dy;
    const int izl = a.iz_first + grp * VPL;   // scan index of this lane's first plane
    const long long r_begin = static_cast<long long>(seg) * a.rows_per_seg;
    const long long r_end = min(r_begin + a.rows_per_seg, a.n_rows);
    const int n_stage = r_end > r_begin ? static_cast<int>((r_end - r_begin + a.ch - 1) / a.ch) : 0;
    const int stage_elems = a.ch * a.n_f;

    float2 pre[PRE];
    auto load = [&](int st) {
        const long long r0 = r_begin + static_cast<long long>(st) * a.ch;
        const int n = static_cast<int>(min(static_cast<long long>(a.ch), r_end - r0)) * a.n_f;
        const float2* src = sw + r0 * a.n_f;
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
            const int e = tid + 256 * j;
            pre[j] = e < n ? src[e] : make_float2(0.f, 0.f);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
            const int e = tid + 256 * j;
            if (e < stage_elems) rows[buf * stage_elems + e] = pre[j];
        }
    };

    float2 vox[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) vox[v] = make_float2(0.f, 0.f);
    if (n_stage > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int st = 0; st < n_stage; ++st) {
        if (st + 1 < n_stage) load(st + 1);   // in flight while this stage is summed
        const float2* L = rows + (st & 1) * stage_elems;
        const long long r0 = r_begin + static_cast<long long>(st) * a.ch;
        const int nr = static_cast<int>(min(static_cast<long long>(a.ch), r_end - r0));
        for (int i = 0; i < nr; ++i) {
            const int r = static_cast<int>(r0 + i);
            const int c = r / a.n_z, m = r - c * a.n_z;   // workgroup-uniform
            const double* ch = chan + 4 * c;
            const double rt2 = (x - ch[0]) * (x - ch[0]) + (y - ch[1]) * (y - ch[1]);
            const double rr2 = (x - ch[2]) * (x - ch[2]) + (y - ch[3]) * (y - ch[3]);
            double D[VPL];
            float2 z[VPL];
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const double dzv = (izl + v - m) * a.dz;
                D[v] = a.mono ? 2.0 * sqrt_dp(rt2 + dzv * dzv) : sqrt_dp(rt2 + dzv * dzv) + sqrt_dp(rr2 + dzv * dzv);
                z[v] = cis_rev(a.dk_rev * D[v]);
            }
            const float2* row = L + i * a.n_f;
            for (int f0 = 0; f0 < a.n_f; f0 += kBpFreqBlock) {
                const int f1 = min(f0 + kBpFreqBlock, a.n_f);
                float2 acc[VPL];
                const float2 top = row[f1 - 1];
#pragma unroll
                for (int v = 0; v < VPL; ++v) acc[v] = top;
#pragma unroll 8
                for (int f = f1 - 2; f >= f0; --f) {
                    const float2 af = row[f];
#pragma unroll
                    for (int v = 0; v < VPL; ++v) {
                        const float2 y0 = acc[v];
                        acc[v].x = fmaf(y0.x, z[v].x, fmaf(-y0.y, z[v].y, af.x));
                        acc[v].y = fmaf(y0.x, z[v].y, fmaf(y0.y, z[v].x, af.y));
                    }
                }
                const double kb_rev = a.k0_rev + f0 * a.dk_rev;
#pragma unroll
                for (int v = 0; v < VPL; ++v) {
                    const float2 e = cis_rev(kb_rev * D[v]);
                    vox[v].x = fmaf(e.x, acc[v].x, fmaf(-e.y, acc[v].y, vox[v].x));
                    vox[v].y = fmaf(e.x, acc[v].y, fmaf(e.y, acc[v].x, vox[v].y));
                }
            }
        }
        if (st + 1 < n_stage) store((st + 1) & 1);   // the other buffer: last read in stage st - 1
        __syncthreads();
    }
    if (px < a.nx && py < a.ny) {
        const size_t npix = static_cast<size_t>(a.nx) * a.ny;
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            const size_t plane = static_cast<size_t>(izl + v - a.iz_out0);
            out[(static_cast<size_t>(seg) * a.nz_out + plane) * npix + static_cast<size_t>(py) * a.nx + px] = vox[v];
        }
    }
}

// image[i] = sum over segments s of part[s][i], in segment order.
__global__ void bp_reduce_kernel(const float2* __restrict__ part, int n_seg, long long n, float2* __restrict__ img) {
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += static_cast<long long>(gridDim.x) * 256) {
        float2 acc = part[i];
        for (int s = 1; s < n_seg; ++s) acc = cadd(acc, part[s * n + i]);
        img[i] = acc;
    }
}

}  // namespace

int launch_simulate(const pl_geometry* g, const DeviceTables& dt, int n_scat, const double* xyz,
                    const double* refl, float2* echo, hipStream_t s) {
    SimArgs a{};
    a.n_ch = g->n_ch;
    a.n_z = g->n_scan;
    a.n_f = g->n_freq;
    a.n_scat = n_scat;
    a.n_chunks = (g->n_freq + kSimChunk - 1) / kSimChunk;
    a.z0 = g->scan_z0;
    a.dz = g->scan_step;
    a.dk = g->n_freq > 1 ? (g->k[g->n_freq - 1] - g->k[0]) / (g->n_freq - 1) : 0.0;
    const long long total = static_cast<long long>(a.n_ch) * a.n_z * a.n_chunks;
    const long long blocks = (total + 255) / 256;
    if (blocks > 0x7fffffffLL) return fail(PL_EUNSUPPORTED, "echo cube too large");
    hipLaunchKernelGGL(simulate_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, dt.chan, dt.k, xyz,
                       refl, a, echo);
    return check_launch("simulate echo");
}

BpLayout bp_layout(const pl_geometry* g, const pl_image_grid* grid, int nz) {
    BpLayout L;
    const long long n_rows = static_cast<long long>(g->n_ch) * g->n_scan;
    const int tiles = ((grid->nx + kBpTile - 1) / kBpTile) * ((grid->ny + kBpTile - 1) / kBpTile);
    const int groups = nz / 4 + (nz % 4) / 2 + (nz % 2);
    L.ch = std::max(1, std::min(32, kBpStageElems / std::max(1, g->n_freq)));
    // segments of the rows so that a thin slab still gives about 2048 workgroups
    const long long base = static_cast<long long>(tiles) * groups;
    long long seg = std::max(1LL, std::min(64LL, (2048 + base - 1) / base));
    seg = std::min(seg, std::max(1LL, n_rows / L.ch));
    long long per = (n_rows + seg - 1) / seg;
    per = (per + L.ch - 1) / L.ch * L.ch;
    L.rows_per_seg = per;
    L.n_seg = static_cast<int>((n_rows + per - 1) / per);
    const size_t weighted = static_cast<size_t>(n_rows) * g->n_freq * 8;
    L.off_part = (weighted + 255) & ~static_cast<size_t>(255);
    L.bytes = L.n_seg > 1 ? L.off_part + static_cast<size_t>(L.n_seg) * nz * grid->nx * grid->ny * 8 : weighted;
    return L;
}

int launch_bp(const pl_geometry* g, const DeviceTables& dt, const pl_image_grid* grid, int iz0, int nz,
              const float2* echo, char* ws, float2* image, hipStream_t s) {
    if (g->n_freq > kBpStageElems) return fail(PL_EUNSUPPORTED, "BP stages at most %d frequencies", kBpStageElems);
    const BpLayout L = bp_layout(g, grid, nz);
    float2* weighted = reinterpret_cast<float2*>(ws);
    const long long total = static_cast<long long>(g->n_ch) * g->n_scan * g->n_freq;
    hipLaunchKernelGGL(weight_echo_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, echo,
                       dt.k, g->n_freq, total, weighted);
    int rc = check_launch("weight echo");
    if (rc) return rc;
    float2* part = L.n_seg > 1 ? reinterpret_cast<float2*>(ws + L.off_part) : image;
    BpArgs a{};
    a.n_ch = g->n_ch;
    a.n_z = g->n_scan;
    a.n_f = g->n_freq;
    a.nx = grid->nx;
    a.ny = grid->ny;
    a.tiles_x = (grid->nx + kBpTile - 1) / kBpTile;
    a.n_tiles = a.tiles_x * ((grid->ny + kBpTile - 1) / kBpTile);
    a.iz_out0 = iz0;
    a.nz_out = nz;
    a.rows_per_seg = static_cast<int>(L.rows_per_seg);
    a.ch = L.ch;
    a.mono = g->mode == PL_MONO;
    a.n_rows = static_cast<long long>(g->n_ch) * g->n_scan;
    a.x0 = grid->x0;
    a.y0 = grid->y0;
    a.dx = grid->dx;
    a.dy = grid->dy;
    a.dz = g->scan_step;
    a.k0_rev = g->k[0] * (0.5 / kPi);
    a.dk_rev = (g->n_freq > 1 ? (g->k[g->n_freq - 1] - g->k[0]) / (g->n_freq - 1) : 0.0) * (0.5 / kPi);
    const size_t smem = 2ull * L.ch * g->n_freq * sizeof(float2);
    // planes in groups of 4, then a pair, then a single plane
    int iz = iz0;
    const int left[3] = {nz / 4, (nz % 4) / 2, nz % 2};
    const int vpl[3] = {4, 2, 1};
    for (int k = 0; k < 3; ++k) {
        if (!left[k]) continue;
        a.iz_first = iz;
        a.n_groups = left[k];
        const long long blocks = static_cast<long long>(a.n_tiles) * a.n_groups * L.n_seg;
        if (blocks > 0x7fffffffLL) return fail(PL_EUNSUPPORTED, "too many voxels");
        if (vpl[k] == 4)
            hipLaunchKernelGGL(bp_tile_kernel<4>, dim3(static_cast<unsigned>(blocks)), dim3(256), smem, s, weighted,
                               dt.chan, a, part);
        else if (vpl[k] == 2)
            hipLaunchKernelGGL(bp_tile_kernel<2>, dim3(static_cast<unsigned>(blocks)), dim3(256), smem, s, weighted,
                               dt.chan, a, part);
        else
            hipLaunchKernelGGL(bp_tile_kernel<1>, dim3(static_cast<unsigned>(blocks)), dim3(256), smem, s, weighted,
                               dt.chan, a, part);
        if ((rc = check_launch("back-projection (BP)"))) return rc;
        iz += vpl[k] * left[k];
    }
    if (L.n_seg > 1) {
        const long long n = static_cast<long long>(nz) * grid->nx * grid->ny;
        const int blocks = static_cast<int>(std::min<long long>((n + 255) / 256, 8192));
        hipLaunchKernelGGL(bp_reduce_kernel, dim3(blocks), dim3(256), 0, s, part, L.n_seg, n, image);
        rc = check_launch("back-projection (BP) segment sum");
    }
    return rc;
}

}  // namespace pl
