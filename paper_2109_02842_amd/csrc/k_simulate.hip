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

struct BpArgs {
    int n_ch, n_z, n_f, nx, ny, iz0, nz, mono;
    double x0, y0, dx, dy, dz, k0, dk;
};

// One thread per voxel (x fastest).  For every (channel, scan position) the
// path D = R_T + R_R (float64) gives the phasors exp(j k_0 D) and
// exp(j dk D); the frequency sum then runs as a phasor recurrence, restarted
// from a direct evaluation every 32 frequencies.  The k_f-weighted echo row
// is the same for every lane of a wavefront.
__global__ __launch_bounds__(256) void bp_kernel(const float2* __restrict__ sw, const double* __restrict__ chan,
                                                 BpArgs a, float2* __restrict__ img) {
    const long long v = blockIdx.x * 256LL + threadIdx.x;
    const long long nvox = static_cast<long long>(a.nx) * a.ny * a.nz;
    if (v >= nvox) return;
    const int ix = static_cast<int>(v % a.nx);
    const int iy = static_cast<int>((v / a.nx) % a.ny);
    const int iz = a.iz0 + static_cast<int>(v / (static_cast<long long>(a.nx) * a.ny));
    const double x = a.x0 + ix * a.dx, y = a.y0 + iy * a.dy;
    const double k0_rev = a.k0 * (0.5 / kPi), dk_rev = a.dk * (0.5 / kPi);
    float2 acc = make_float2(0.f, 0.f);
    for (int c = 0; c < a.n_ch; ++c) {
        const double* ch = chan + 4 * c;
        const double rt2 = (x - ch[0]) * (x - ch[0]) + (y - ch[1]) * (y - ch[1]);
        const double rr2 = (x - ch[2]) * (x - ch[2]) + (y - ch[3]) * (y - ch[3]);
        for (int m = 0; m < a.n_z; ++m) {
            const double dzv = (iz - m) * a.dz;
            const double d = a.mono ? 2.0 * sqrt(rt2 + dzv * dzv) : sqrt(rt2 + dzv * dzv) + sqrt(rr2 + dzv * dzv);
            const float2* row = sw + (static_cast<size_t>(c) * a.n_z + m) * a.n_f;
            const float2 st = cis_rev(dk_rev * d);
            for (int f0 = 0; f0 < a.n_f; f0 += 32) {
                float2 ph = cis_rev((k0_rev + f0 * dk_rev) * d);
                const int n = min(32, a.n_f - f0);
                for (int f = 0; f < n; ++f) {
                    const float2 s = row[f0 + f];
                    acc.x += s.x * ph.x - s.y * ph.y;
                    acc.y += s.x * ph.y + s.y * ph.x;
                    ph = cmul(ph, st);
                }
            }
        }
    }
    img[v] = acc;
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

int launch_bp(const pl_geometry* g, const DeviceTables& dt, const pl_image_grid* grid, int iz0, int nz,
              const float2* echo, float2* weighted, float2* image, hipStream_t s) {
    const long long total = static_cast<long long>(g->n_ch) * g->n_scan * g->n_freq;
    hipLaunchKernelGGL(weight_echo_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, echo,
                       dt.k, g->n_freq, total, weighted);
    int rc = check_launch("weight echo");
    if (rc) return rc;
    BpArgs a{};
    a.n_ch = g->n_ch;
    a.n_z = g->n_scan;
    a.n_f = g->n_freq;
    a.nx = grid->nx;
    a.ny = grid->ny;
    a.iz0 = iz0;
    a.nz = nz;
    a.mono = g->mode == PL_MONO;
    a.x0 = grid->x0;
    a.y0 = grid->y0;
    a.dx = grid->dx;
    a.dy = grid->dy;
    a.dz = g->scan_step;
    a.k0 = g->k[0];
    a.dk = g->n_freq > 1 ? (g->k[g->n_freq - 1] - g->k[0]) / (g->n_freq - 1) : 0.0;
    const long long nvox = static_cast<long long>(grid->nx) * grid->ny * nz;
    const long long blocks = (nvox + 255) / 256;
    if (blocks > 0x7fffffffLL) return fail(PL_EUNSUPPORTED, "too many voxels");
    hipLaunchKernelGGL(bp_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, weighted, dt.chan, a, image);
    return check_launch("back-projection (BP)");
}

}  // namespace pl
