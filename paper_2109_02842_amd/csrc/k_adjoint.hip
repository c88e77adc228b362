// Adjoint of the range compression (the type-2 transform of eq. 8a / 19a):
//   S~[c][kz][f] = w[kz][f] sum_i q~[c][kz][i] exp(-j k'[kz][f] (l_lo[c] + i du)),
// the transpose of q[c][kz][i] = sum_f w[kz][f] S[c][kz][f] exp(+j k' l_i).
// For fine grids of N = 64 R points the forward NUFFT runs on the wavefront
// FFT and range_adjoint_wave_kernel is its exact transpose (the same
// spreading kernel, deapodisation and grid).  Otherwise the sums are direct
// (range_adjoint_kernel): one wavefront per (c, kz), lanes over frequencies,
// the profile read 64 samples per coalesced load and broadcast by readlane,
// the phasor advanced by a recurrence in FP32 and re-anchored from an
// FP64-reduced phase every 32 samples.
//
// Also the adjoint of the interpolated back-projection (A4 transposed), the
// owner-computes scatter described at backproject_adjoint_kernel.
#include <cstring>

#include "device.hpp"

namespace pl {
namespace {

struct RangeAdjArgs {
    int n_ch, n_z, n_f, n_l;
    double du;
};

__global__ __launch_bounds__(256) void range_adjoint_kernel(const float2* __restrict__ qt,
                                                            const double* __restrict__ llo,
                                                            const double* __restrict__ kp,
                                                            const float* __restrict__ wk, RangeAdjArgs a,
                                                            float2* __restrict__ St) {
    const long long pair = static_cast<long long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (pair >= static_cast<long long>(a.n_ch) * a.n_z) return;  // no barriers in this kernel
    const int lane = threadIdx.x & 63;
    const int c = static_cast<int>(pair / a.n_z), kz = static_cast<int>(pair - static_cast<long long>(c) * a.n_z);
    const float2* row = qt + pair * a.n_l;
    const double l0 = llo[c];
    for (int f0 = 0; f0 < a.n_f; f0 += 64) {
        const int f = f0 + lane;
        const bool fok = f < a.n_f;
        const double k = fok ? kp[static_cast<size_t>(kz) * a.n_f + f] : 0.0;
        const float w = fok ? wk[static_cast<size_t>(kz) * a.n_f + f] : 0.f;
        const double rev = -k * (0.5 / kPi);  // phase in revolutions per metre
        const float2 d = cis_rev(rev * a.du);
        float2 acc = make_float2(0.f, 0.f), ph = make_float2(1.f, 0.f);
        // 64 range samples per coalesced load, broadcast to the lanes by readlane
        for (int ib = 0; ib < a.n_l; ib += 64) {
            const float2 qv = ib + lane < a.n_l ? row[ib + lane] : make_float2(0.f, 0.f);
            const int nb = min(64, a.n_l - ib);
            for (int j = 0; j < nb; ++j) {
                if ((j & 31) == 0) ph = cis_rev(rev * (l0 + (ib + j) * a.du));
                const float qx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qv.x), j));
                const float qy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qv.y), j));
                acc.x += ph.x * qx - ph.y * qy;
                acc.y += ph.x * qy + ph.y * qx;
                ph = cmul(ph, d);
            }
        }
        if (fok) St[pair * a.n_f + f] = make_float2(w * acc.x, w * acc.y);
    }
}

struct RangeAdjWaveArgs {
    int n_z, n_f, n_l, pad_;
    double du, h, beta, inv_h;
};

// The transpose, step by step in reverse, of nufft_wave_kernel: the profile
// times the deapodisation, placed at its fine-grid cells (the crop
// transposed), the forward FFT (the conjugate transpose of the unnormalised
// inverse one) as conj(IFFT(conj b)), then each frequency gathers the cells
// its kernel spread into (the spreading transposed) and takes the conjugate
// strength factor w exp(-j k' l_mid).  The last FFT pass leaves X[k] in the
// slot its butterfly read, row k mod R, 9 m1 + m2 with k / R = m1 + 8 m2.
template <int R>
__global__ __launch_bounds__(64) void range_adjoint_wave_kernel(const float2* __restrict__ qt,
                                                               const double* __restrict__ llo,
                                                               const double* __restrict__ kp,
                                                               const float* __restrict__ wk,
                                                               const float2* __restrict__ tw,
                                                               const float* __restrict__ deap, RangeAdjWaveArgs a,
                                                               float2* __restrict__ St) {
    constexpr int N = 64 * R;
    extern __shared__ float2 smem_f2[];
    float2* A = smem_f2;   // R rows of kWaveRow
    const int lane = threadIdx.x;
    const int pair = blockIdx.x;   // = c * n_z + kap
    const int c = pair / a.n_z;
    const int kap = pair - c * a.n_z;
    const float2* row = qt + static_cast<size_t>(pair) * a.n_l;
    const int half = a.n_l / 2;
#pragma unroll
    for (int j = 0; j < R; ++j) A[64 * j + lane] = make_float2(0.f, 0.f);
    wave_lds_sync();
    for (int i = lane; i < a.n_l; i += 64) {
        const float2 v = row[i];
        const float d = deap[i];
        const int k = i < half ? i - half + N : i - half;
        A[k] = make_float2(v.x * d, -v.y * d);   // conjugated
    }
    wave_lds_sync();
    wave_ifft<R>(A, tw, lane, [&](int k, float2 v) {
        const int k1 = k % R, k2 = k / R;
        A[k1 * kWaveRow + 9 * (k2 & 7) + (k2 >> 3)] = v;
    });
    wave_lds_sync();

    const double lmid = llo[c] + half * a.du;
    const double cell = a.du * N * (0.5 / kPi);
    for (int fb = 0; fb < a.n_f; fb += 64) {
        const int f = fb + lane;
        if (f >= a.n_f) continue;
        const float w = wk[static_cast<size_t>(kap) * a.n_f + f];
        float2 res = make_float2(0.f, 0.f);
        if (w != 0.0f) {
            const double kpf = kp[static_cast<size_t>(kap) * a.n_f + f];
            const double y = kpf * cell;
            // the cells with -h < k - y < h, as in the spreading
            const int k_lo = static_cast<int>(floor(y - a.h)) + 1;
            const int k_hi = static_cast<int>(ceil(y + a.h)) - 1;
            float2 acc = make_float2(0.f, 0.f);
            for (int k = k_lo; k <= k_hi; ++k) {
                const float z = static_cast<float>((k - y) * a.inv_h);
                const float phi = __expf(static_cast<float>(a.beta) * (__builtin_amdgcn_sqrtf(fmaxf(1.f - z * z, 0.f)) - 1.f));
                const int kk = k < 0 ? k + N : (k >= N ? k - N : k);
                const int k1 = kk % R, k2 = kk / R;
                const float2 b = A[k1 * kWaveRow + 9 * (k2 & 7) + (k2 >> 3)];
                acc.x += b.x * phi;   // conj(X[k]) phi
                acc.y -= b.y * phi;
            }
            const float2 ph = cis(-kpf * lmid);
            res = cscale(cmul(acc, ph), w);
        }
        St[static_cast<size_t>(pair) * a.n_f + f] = res;
    }
}

template <int R>
int launch_range_adjoint_wave(const HybridPlan& p, const float2* qt, char* ws, float2* St, hipStream_t s) {
    RangeAdjWaveArgs a{};
    a.n_z = p.n_z;
    a.n_f = p.n_f;
    a.n_l = p.n_l;
    a.du = p.du;
    a.h = p.h;
    a.inv_h = 1.0 / p.h;
    a.beta = p.beta;
    const long long pairs = static_cast<long long>(p.n_ch) * p.n_z;
    if (pairs > 0x7fffffffLL) return fail(PL_EUNSUPPORTED, "range adjoint: too many (channel, k_z) pairs");
    const size_t smem = 8ull * R * kWaveRow;
    auto fn = range_adjoint_wave_kernel<R>;
    if (smem > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            static_cast<int>(smem)) != hipSuccess)
        return fail(PL_EDEVICE, "range adjoint: LDS of %zu bytes refused", smem);
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(pairs)), dim3(64), smem, s, qt,
                       reinterpret_cast<const double*>(ws + p.off_llo), reinterpret_cast<const double*>(ws + p.off_kp),
                       reinterpret_cast<const float*>(ws + p.off_wk), reinterpret_cast<const float2*>(ws + p.off_tw_fine),
                       reinterpret_cast<const float*>(ws + p.off_deap), a, St);
    return check_launch("range compression (adjoint, wavefront per pair)");
}

// Adjoint of the back-projection (the transpose of A4):
//   q~[c][kz][i] = sum_p sum_j [i = floor(u_c(p)) - 1 + j] w_j(p, c)
//                  conj(exp(j k_ref l_c(p))) G~[p][kz].
// Owner computes: one workgroup = one channel c x one block of KB k_z bins x
// one segment of S range samples; every element of q~ is written once, by
// one workgroup, with no atomics and no zero fill beforehand.  The
// workgroup lists, in tile order, the 8x8 pixel tiles whose range interval
// (lower bound: distance to the tile's rectangle; upper: its farthest
// corner) can reach the segment; wavefront w takes list entries w, w+4, ...
// Its lanes set up the tile's 64 pixels (first tap, four weights, carrier),
// then the wavefront walks the pixels in order with the pixel's values
// broadcast by readlane and its lanes over k_z bins (KB = 32: a lane per k_z
// bin and real/imaginary part; KB = 64: a lane per bin, both parts), adding
// each tap inside the segment into the wavefront's own LDS copy of the
// segment (plain read-modify-write: a lane owns its address).  The four
// copies are summed in a fixed order at the end, so the result is the same
// bit for bit on every run.
struct AdjArgs {
    int n_ch, n_z, n_l, nx, ny, tiles_x, n_tiles, n_seg, n_work, per_xcd;
    double x0, y0, dx, dy, inv_du;
    float coef[4][4];
    double kref[kMaxBlocks];
};

constexpr int kAdjWaves = 4;

__device__ __forceinline__ double rect_dist(double px, double py, double x0, double x1, double y0, double y1) {
    const double cx = fmin(fmax(px, x0), x1), cy = fmin(fmax(py, y0), y1);
    return sqrt((px - cx) * (px - cx) + (py - cy) * (py - cy));
}

template <int KB>
constexpr int adj_segment() { return KB == 32 ? 32 : 16; }
// floats of one wavefront's copy: [2 parts][KB rows][S + 1]
template <int KB>
constexpr int adj_copy_floats() { return 2 * KB * (adj_segment<KB>() + 1); }

template <int KB>
__global__ __launch_bounds__(64 * kAdjWaves) void backproject_adjoint_kernel(const float2* __restrict__ Gt,
                                                                           const double* __restrict__ chan,
                                                                           const double* __restrict__ llo,
                                                                           AdjArgs a, float2* __restrict__ qt) {
    constexpr int S = adj_segment<KB>();
    constexpr int LR = S + 1;            // floats per row (odd: the rows of one column fall in distinct banks)
    constexpr int PL = KB * LR;          // floats per part plane
    constexpr int CF = adj_copy_floats<KB>();
    constexpr int NT = 64 * kAdjWaves;
    extern __shared__ float acc[];       // [kAdjWaves][2][KB][LR]
    __shared__ int tiles[NT];
    __shared__ int wcount[kAdjWaves];

    const int work = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    if (work >= a.n_work) return;  // workgroup-uniform, before any barrier
    const int c = work % a.n_ch;
    const int rest = work / a.n_ch;
    const int seg = rest % a.n_seg;
    const int blk = rest / a.n_seg;
    const int s0 = seg * S;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double xT = chan[4 * c], yT = chan[4 * c + 1], xR = chan[4 * c + 2], yR = chan[4 * c + 3];
    const double l0 = llo[c];
    const double kref_rev = a.kref[blk] * (0.5 / kPi);

    for (int e = tid; e < kAdjWaves * CF; e += NT) acc[e] = 0.f;

    // this lane's k_z bin and part(s)
    const int kl = KB == 32 ? (lane & 31) : lane;
    const int part = KB == 32 ? (lane >> 5) : 0;
    const int kz = blk * KB + kl;
    const bool kok = kz < a.n_z;
    float* mine = acc + wave * CF + part * PL + kl * LR;

#pragma unroll 1
    for (int t0 = 0; t0 < a.n_tiles; t0 += NT) {
        bool hit = false;
        const int t = t0 + tid;
        if (t < a.n_tiles) {
            const int tx0 = (t % a.tiles_x) * 8, ty0 = (t / a.tiles_x) * 8;
            const double xa = a.x0 + tx0 * a.dx, xb = a.x0 + min(tx0 + 7, a.nx - 1) * a.dx;
            const double ya = a.y0 + ty0 * a.dy, yb = a.y0 + min(ty0 + 7, a.ny - 1) * a.dy;
            const double lmin = rect_dist(xT, yT, xa, xb, ya, yb) + rect_dist(xR, yR, xa, xb, ya, yb);
            double lmax = 0.0;
            for (int k = 0; k < 4; ++k) {
                const double x = (k & 1) ? xb : xa, y = (k & 2) ? yb : ya;
                lmax = fmax(lmax, sqrt((x - xT) * (x - xT) + (y - yT) * (y - yT)) +
                                      sqrt((x - xR) * (x - xR) + (y - yR) * (y - yR)));
            }
            // taps floor(u) - 1 .. floor(u) + 2 reach [s0, s0 + S) only if
            // s0 - 2 <= u < s0 + S + 1
            const double umin = (lmin - l0) * a.inv_du, umax = (lmax - l0) * a.inv_du;
            hit = umax >= s0 - 3.0 && umin <= s0 + S + 1.0;
        }
        // ordered compaction of the hits: within the wavefront by ballot,
        // across wavefronts by their counts
        const unsigned long long bal = __ballot(hit);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wave] = __popcll(bal);
        __syncthreads();
        int base = 0, nl = 0;
        for (int w = 0; w < kAdjWaves; ++w) {
            base += w < wave ? wcount[w] : 0;
            nl += wcount[w];
        }
        if (hit) tiles[base + below] = t;
        __syncthreads();
#pragma unroll 1
        for (int k = wave; k < nl; k += kAdjWaves) {
            const int tt = tiles[k];
            const int px = (tt % a.tiles_x) * 8 + (lane & 7), py = (tt / a.tiles_x) * 8 + (lane >> 3);
            // this lane's pixel: first tap relative to the segment, weights, conj carrier
            int i0 = -1000000, pix = 0;
            float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f, cr = 0.f, ci = 0.f;
            if (px < a.nx && py < a.ny) {
                const double xg = a.x0 + px * a.dx, yg = a.y0 + py * a.dy;
                const double l = sqrt((xg - xT) * (xg - xT) + (yg - yT) * (yg - yT)) +
                                 sqrt((xg - xR) * (xg - xR) + (yg - yR) * (yg - yR));
                const double u = (l - l0) * a.inv_du;
                const double fl = floor(u);
                const float tt2 = static_cast<float>(u - fl);
                w0 = ((a.coef[0][3] * tt2 + a.coef[0][2]) * tt2 + a.coef[0][1]) * tt2 + a.coef[0][0];
                w1 = ((a.coef[1][3] * tt2 + a.coef[1][2]) * tt2 + a.coef[1][1]) * tt2 + a.coef[1][0];
                w2 = ((a.coef[2][3] * tt2 + a.coef[2][2]) * tt2 + a.coef[2][1]) * tt2 + a.coef[2][0];
                w3 = ((a.coef[3][3] * tt2 + a.coef[3][2]) * tt2 + a.coef[3][1]) * tt2 + a.coef[3][0];
                const float2 car = cis_rev(kref_rev * l);
                cr = car.x;
                ci = car.y;
                i0 = static_cast<int>(fl) - 1 - s0;
                pix = py * a.nx + px;
            }
#pragma unroll 1
            for (int g0 = 0; g0 < 64; g0 += 16) {
                // the group's G~ values first (one load per pixel and lane),
                // so their latency is paid once per 16 pixels
                float2 gv[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int ppix = __builtin_amdgcn_readlane(pix, g0 + q);  // 0 for pixels off the grid
                    gv[q] = kok ? Gt[static_cast<size_t>(ppix) * a.n_z + kz] : make_float2(0.f, 0.f);
                }
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int p = g0 + q;
                    const int pi0 = __builtin_amdgcn_readlane(i0, p);
                    if (pi0 < -3 || pi0 >= S) continue;  // wavefront-uniform
                    const float pcr = rdl(cr, p), pci = rdl(ci, p);
                    const float pw[4] = {rdl(w0, p), rdl(w1, p), rdl(w2, p), rdl(w3, p)};
                    // conj(carrier) * G~
                    const float hr = pcr * gv[q].x + pci * gv[q].y, hi = pcr * gv[q].y - pci * gv[q].x;
                    const float h = part ? hi : hr;
                    if (pi0 >= 0 && pi0 + 3 < S) {
                        // all four taps in the segment: one batch of reads,
                        // one wait, one batch of writes
                        float* r = mine + pi0;
                        if (KB == 32) {
                            const float v0 = r[0], v1 = r[1], v2 = r[2], v3 = r[3];
                            r[0] = v0 + pw[0] * h;
                            r[1] = v1 + pw[1] * h;
                            r[2] = v2 + pw[2] * h;
                            r[3] = v3 + pw[3] * h;
                        } else {
                            const float v0 = r[0], v1 = r[1], v2 = r[2], v3 = r[3];
                            const float u0 = r[PL], u1 = r[PL + 1], u2 = r[PL + 2], u3 = r[PL + 3];
                            r[0] = v0 + pw[0] * hr;
                            r[1] = v1 + pw[1] * hr;
                            r[2] = v2 + pw[2] * hr;
                            r[3] = v3 + pw[3] * hr;
                            r[PL] = u0 + pw[0] * hi;
                            r[PL + 1] = u1 + pw[1] * hi;
                            r[PL + 2] = u2 + pw[2] * hi;
                            r[PL + 3] = u3 + pw[3] * hi;
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int i = pi0 + j;
                            if (i >= 0 && i < S) {
                                if (KB == 32) {
                                    mine[i] += pw[j] * h;
                                } else {
                                    mine[i] += pw[j] * hr;
                                    mine[PL + i] += pw[j] * hi;
                                }
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();  // the tile list is rebuilt next
    }
    const int n_s = min(S, a.n_l - s0);
    float2* dst = qt + static_cast<size_t>(c) * a.n_z * a.n_l + s0;
    for (int e = tid; e < KB * S; e += NT) {
        const int r = e / S, i = e - r * S;
        const int kzr = blk * KB + r;
        if (kzr < a.n_z && i < n_s) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int w = 0; w < kAdjWaves; ++w) {
                re += acc[w * CF + r * LR + i];
                im += acc[w * CF + PL + r * LR + i];
            }
            dst[static_cast<size_t>(kzr) * a.n_l + i] = make_float2(re, im);
        }
    }
}

template <int KB>
int launch_adjoint_cfg(const AdjArgs& a, unsigned blocks, hipStream_t s, const float2* Gt, const double* chan,
                       const double* llo, float2* qt) {
    auto fn = backproject_adjoint_kernel<KB>;
    const size_t smem = static_cast<size_t>(kAdjWaves) * adj_copy_floats<KB>() * sizeof(float);
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem));
    if (e != hipSuccess) return fail(PL_EDEVICE, "adjoint back-projection LDS of %zu bytes: %s", smem, hipGetErrorString(e));
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * kAdjWaves), smem, s, Gt, chan, llo, a, qt);
    return check_launch("adjoint back-projection");
}

}  // namespace

int launch_range_adjoint(const HybridPlan& p, const float2* qt, char* ws, float2* St, hipStream_t s) {
    if (p.n_fine % 64 == 0) {
        switch (p.n_fine / 64) {
#define PL_RA(R) \
            case R: return launch_range_adjoint_wave<R>(p, qt, ws, St, s);
            PL_RA(2) PL_RA(3) PL_RA(4) PL_RA(5) PL_RA(6) PL_RA(8) PL_RA(9) PL_RA(10) PL_RA(12) PL_RA(15) PL_RA(16)
            PL_RA(18) PL_RA(20) PL_RA(24) PL_RA(25) PL_RA(27) PL_RA(30) PL_RA(32)
#undef PL_RA
            default: break;
        }
    }
    RangeAdjArgs a{};
    a.n_ch = p.n_ch;
    a.n_z = p.n_z;
    a.n_f = p.n_f;
    a.n_l = p.n_l;
    a.du = p.du;
    const long long pairs = static_cast<long long>(p.n_ch) * p.n_z;
    const long long blocks = (pairs + 3) / 4;
    if (blocks > (1LL << 31) - 1) return fail(PL_EUNSUPPORTED, "range adjoint: too many (channel, k_z) pairs");
    hipLaunchKernelGGL(range_adjoint_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, qt,
                       reinterpret_cast<const double*>(ws + p.off_llo), reinterpret_cast<const double*>(ws + p.off_kp),
                       reinterpret_cast<const float*>(ws + p.off_wk), a, St);
    return check_launch("range compression (adjoint)");
}


int launch_backproject_adjoint(const HybridPlan& p, const DeviceTables& dt, const float2* Gt, char* ws, float2* qt,
                               hipStream_t s) {
    if (p.block != 32 && p.block != 64)
        return fail(PL_EUNSUPPORTED, "adjoint back-projection takes 32 or 64 k_z bins per block");
    AdjArgs a{};
    a.n_ch = p.n_ch;
    a.n_z = p.n_z;
    a.n_l = p.n_l;
    a.nx = p.nx;
    a.ny = p.ny;
    a.tiles_x = (p.nx + 7) / 8;
    a.n_tiles = a.tiles_x * ((p.ny + 7) / 8);
    const int S = p.block == 32 ? adj_segment<32>() : adj_segment<64>();
    a.n_seg = (p.n_l + S - 1) / S;
    const long long work = static_cast<long long>(p.n_ch) * p.n_blocks * a.n_seg;
    if (work > (1LL << 30)) return fail(PL_EUNSUPPORTED, "adjoint back-projection: too many work items");
    a.n_work = static_cast<int>(work);
    a.per_xcd = (a.n_work + 7) / 8;
    a.x0 = p.x0;
    a.y0 = p.y0;
    a.dx = p.dx;
    a.dy = p.dy;
    a.inv_du = 1.0 / p.du;
    std::memcpy(a.coef, p.coef, sizeof(a.coef));
    for (int b = 0; b < kMaxBlocks; ++b) a.kref[b] = p.kref[b];
    const unsigned blocks = static_cast<unsigned>(8 * a.per_xcd);
    const double* llo = reinterpret_cast<const double*>(ws + p.off_llo);
    return p.block == 32 ? launch_adjoint_cfg<32>(a, blocks, s, Gt, dt.chan, llo, qt)
                         : launch_adjoint_cfg<64>(a, blocks, s, Gt, dt.chan, llo, qt);
}

}  // namespace pl
