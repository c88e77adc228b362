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
// Owner computes: one workgroup = one channel c x 64 k_z bins x one segment
// [s0, s0 + S) of the range grid; every element of q~ is written once, by
// one workgroup, with no atomics and no zero fill beforehand.  The
// workgroup lists, in tile order, the 8x8 pixel tiles whose range interval
// (lower bound: distance to the tile's rectangle; upper: its farthest
// corner) can reach the segment; wavefront w takes list entries w, w+4, ...
// For a tile, lane = pixel: its first tap relative to the segment, four
// weights and carrier (one per plan block of k_z bins the workgroup
// covers); the pixels whose taps reach the segment are ranked by first tap
// (ties in lane order) and their records written to the wavefront's LDS in
// that order.  Then lane = k_z bin: the wavefront walks the ranked pixels,
// each record read by broadcast, and adds w_j conj(c) G~[p][kz] into four
// complex accumulators for the samples cur .. cur + 3; once the next pixel's
// first tap is past cur, the first of them goes into the lane's register
// copy of the segment at cur and the window moves on.  A tile thus costs one
// register-indexed update per sample it reaches, not four per pixel.  The
// four wavefronts' copies are summed through LDS in a fixed order, so the
// result is the same bit for bit on every run.
struct AdjArgs {
    int n_ch, n_z, n_l, nx, ny, tiles_x, n_tiles, n_seg, n_work, per_xcd, block;
    double x0, y0, dx, dy, inv_du;
    float coef[4][4];
    double kref[kMaxBlocks];
};

constexpr int kAdjWaves = 4;
constexpr int kAdjSeg = 32;    // range samples per workgroup
constexpr int kAdjBins = 64;   // k_z bins per workgroup, one per lane

// G~ through a buffer descriptor: the pixel's row offset is scalar, the
// lane's bin a fixed per-lane offset, and a lane past the last bin reads
// beyond the descriptor (zero) instead of branching.
typedef unsigned int adj_u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t adj_rsrc(const float2* p, unsigned bytes) {
    const unsigned long long a = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
    void* u = reinterpret_cast<void*>((static_cast<unsigned long long>(hi) << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(u, 0, __builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

__device__ __forceinline__ double rect_dist(double px, double py, double x0, double x1, double y0, double y1) {
    const double cx = fmin(fmax(px, x0), x1), cy = fmin(fmax(py, y0), y1);
    return sqrt((px - cx) * (px - cx) + (py - cy) * (py - cy));
}

__global__ __launch_bounds__(64 * kAdjWaves) void backproject_adjoint_kernel(const float2* __restrict__ Gt,
                                                                           const double* __restrict__ chan,
                                                                           const double* __restrict__ llo,
                                                                           AdjArgs a, float2* __restrict__ qt) {
    constexpr int S = kAdjSeg, NW = kAdjWaves, NT = 64 * NW;
    __shared__ int tiles[NT];
    __shared__ int wcount[NW];
    // the ranked pixels of a tile, per wavefront: tap weights, the carriers
    // of bins [0, 32) and [32, 64) of the workgroup, (pixel, first tap
    // relative to the segment)
    __shared__ float4 rw[NW][64];
    __shared__ float2 rc[NW][2][64];
    __shared__ int2 rpi[NW][64];
    __shared__ float sum_re[S][65], sum_im[S][65];   // odd row length: a lane per bank

    const int work = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    if (work >= a.n_work) return;  // workgroup-uniform, before any barrier
    const int c = work % a.n_ch;
    const int rest = work / a.n_ch;
    const int seg = rest % a.n_seg;
    const int kb = rest / a.n_seg;
    const int s0 = seg * S;
    const int kz0 = kb * kAdjBins;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double xT = chan[4 * c], yT = chan[4 * c + 1], xR = chan[4 * c + 2], yR = chan[4 * c + 3];
    const double l0 = llo[c];
    // the plan's reference wavenumbers of the workgroup's two halves of bins
    const double kr0 = a.kref[kz0 / a.block] * (0.5 / kPi);
    const double kr1 = a.kref[min(kz0 + 32, a.n_z - 1) / a.block] * (0.5 / kPi);
    const int kz = kz0 + lane;
    const bool kok = kz < a.n_z;
    float4* myw = rw[wave];
    float2* myc = rc[wave][lane >> 5];   // this lane's half of the bins
    int2* mypi = rpi[wave];
    const __amdgpu_buffer_rsrc_t grs =
        adj_rsrc(Gt, static_cast<unsigned>(static_cast<size_t>(a.nx) * a.ny * a.n_z * sizeof(float2)));
    const unsigned gvoff = kok ? static_cast<unsigned>(kz) * 8u : 0x80000000u;

    // the lane's copy of the segment, real and imaginary parts apart (each
    // array stays in registers under a wavefront-uniform index)
    float acr[S], aci[S];
#pragma unroll
    for (int i = 0; i < S; ++i) acr[i] = aci[i] = 0.f;

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
        for (int w = 0; w < NW; ++w) {
            base += w < wave ? wcount[w] : 0;
            nl += wcount[w];
        }
        if (hit) tiles[base + below] = t;
        __syncthreads();
#pragma unroll 1
        for (int k = wave; k < nl; k += NW) {
            const int tt = tiles[k];
            // lane = pixel of the tile
            const int px = (tt % a.tiles_x) * 8 + (lane & 7), py = (tt / a.tiles_x) * 8 + (lane >> 3);
            int i0 = 1 << 20, pix = 0;
            float4 rwv = make_float4(0.f, 0.f, 0.f, 0.f);
            float2 c0 = make_float2(0.f, 0.f), c1 = c0;
            if (px < a.nx && py < a.ny) {
                const double xg = a.x0 + px * a.dx, yg = a.y0 + py * a.dy;
                const double l = sqrt((xg - xT) * (xg - xT) + (yg - yT) * (yg - yT)) +
                                 sqrt((xg - xR) * (xg - xR) + (yg - yR) * (yg - yR));
                const double u = (l - l0) * a.inv_du;
                const double fl = floor(u);
                const float tf = static_cast<float>(u - fl);
                rwv.x = ((a.coef[0][3] * tf + a.coef[0][2]) * tf + a.coef[0][1]) * tf + a.coef[0][0];
                rwv.y = ((a.coef[1][3] * tf + a.coef[1][2]) * tf + a.coef[1][1]) * tf + a.coef[1][0];
                rwv.z = ((a.coef[2][3] * tf + a.coef[2][2]) * tf + a.coef[2][1]) * tf + a.coef[2][0];
                rwv.w = ((a.coef[3][3] * tf + a.coef[3][2]) * tf + a.coef[3][1]) * tf + a.coef[3][0];
                c0 = cis_rev(kr0 * l);
                c1 = cis_rev(kr1 * l);
                i0 = static_cast<int>(fl) - 1 - s0;
                pix = py * a.nx + px;
            }
            const bool valid = i0 >= -3 && i0 < S;
            const unsigned long long vm = __ballot(valid);
            const int n = __popcll(vm);
            if (n == 0) continue;  // wavefront-uniform
            // rank by first tap, ties in lane order: the smallest tap first,
            // then one ballot per tap value up to the largest
            int vmin = valid ? i0 : S;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) vmin = min(vmin, __shfl_xor(vmin, o));
            vmin = __builtin_amdgcn_readfirstlane(vmin);
            int rank = 0, placed = 0;
#pragma unroll 1
            for (int v = vmin; placed < n; ++v) {
                const unsigned long long m = __ballot(valid && i0 == v);
                if (valid && i0 == v) rank = placed + __popcll(m & ((1ull << lane) - 1ull));
                placed += __popcll(m);
            }
            if (valid) {
                myw[rank] = rwv;
                rc[wave][0][rank] = c0;
                rc[wave][1][rank] = c1;
                mypi[rank] = make_int2(pix, i0);
            }
            wave_lds_sync();   // the records, written by their lanes, read by every lane below

            // lane = k_z bin: walk the ranked pixels
            float2 a0 = make_float2(0.f, 0.f), a1 = a0, a2 = a0, a3 = a0;
            int cur = __builtin_amdgcn_readfirstlane(mypi[0].y);
#pragma unroll 1
            for (int q0 = 0; q0 < n; q0 += 8) {
                // the next eight pixels' G~ first, so their latency is paid
                // once (entries past n hold an earlier tile's pixels or
                // nothing: what they load is never used, and a row offset
                // past G~ reads zeros)
                adj_u32x2 gv[8];
#pragma unroll
                for (int qq = 0; qq < 8; ++qq) {
                    const unsigned pix = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(mypi[q0 + qq].x));
                    gv[qq] = __builtin_amdgcn_raw_buffer_load_b64(grs, gvoff, pix * static_cast<unsigned>(a.n_z) * 8u, 0);
                }
#pragma unroll
                for (int qq = 0; qq < 8; ++qq) {
                    if (q0 + qq >= n) break;  // wavefront-uniform
                    const int pi0 = __builtin_amdgcn_readfirstlane(mypi[q0 + qq].y);
                    while (cur < pi0) {  // samples before this pixel's first tap are complete
                        if (cur >= 0 && cur < S) {
                            acr[cur] += a0.x;
                            aci[cur] += a0.y;
                        }
                        a0 = a1;
                        a1 = a2;
                        a2 = a3;
                        a3 = make_float2(0.f, 0.f);
                        ++cur;
                    }
                    const float4 w = myw[q0 + qq];
                    const float2 car = myc[q0 + qq];
                    const float gr = __uint_as_float(gv[qq].x), gi = __uint_as_float(gv[qq].y);
                    // conj(carrier) * G~
                    const float hr = car.x * gr + car.y * gi, hi = car.x * gi - car.y * gr;
                    a0.x = fmaf(w.x, hr, a0.x);
                    a0.y = fmaf(w.x, hi, a0.y);
                    a1.x = fmaf(w.y, hr, a1.x);
                    a1.y = fmaf(w.y, hi, a1.y);
                    a2.x = fmaf(w.z, hr, a2.x);
                    a2.y = fmaf(w.z, hi, a2.y);
                    a3.x = fmaf(w.w, hr, a3.x);
                    a3.y = fmaf(w.w, hi, a3.y);
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {   // the last pixel's four samples
                if (cur >= 0 && cur < S) {
                    acr[cur] += a0.x;
                    aci[cur] += a0.y;
                }
                a0 = a1;
                a1 = a2;
                a2 = a3;
                ++cur;
            }
            wave_lds_sync();   // every lane has read the records before the next tile's are written
        }
        __syncthreads();  // the tile list is rebuilt next
    }

    // the wavefronts' copies, summed in wavefront order
#pragma unroll 1
    for (int w = 0; w < NW; ++w) {
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < S; ++i) {
                sum_re[i][lane] = (w == 0 ? 0.f : sum_re[i][lane]) + acr[i];
                sum_im[i][lane] = (w == 0 ? 0.f : sum_im[i][lane]) + aci[i];
            }
        }
        __syncthreads();
    }
    const int n_s = min(S, a.n_l - s0);
    for (int e = tid; e < kAdjBins * S; e += NT) {
        const int r = e / S, i = e - r * S;
        const int kzr = kz0 + r;
        if (kzr < a.n_z && i < n_s)
            qt[(static_cast<size_t>(c) * a.n_z + kzr) * a.n_l + s0 + i] = make_float2(sum_re[i][r], sum_im[i][r]);
    }
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
    a.n_seg = (p.n_l + kAdjSeg - 1) / kAdjSeg;
    a.block = p.block;
    const long long bins = (p.n_z + kAdjBins - 1) / kAdjBins;
    const long long work = static_cast<long long>(p.n_ch) * bins * a.n_seg;
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
    // G~ is read through one buffer descriptor (32-bit offsets)
    if (static_cast<unsigned long long>(p.nx) * p.ny * p.n_z * 8 >= (1ull << 31))
        return fail(PL_EUNSUPPORTED, "adjoint back-projection: the spectrum exceeds 2 GiB");
    const unsigned blocks = static_cast<unsigned>(8 * a.per_xcd);
    const double* llo = reinterpret_cast<const double*>(ws + p.off_llo);
    hipLaunchKernelGGL(backproject_adjoint_kernel, dim3(blocks), dim3(64 * kAdjWaves), 0, s, Gt, dt.chan, llo, a, qt);
    return check_launch("adjoint back-projection");
}

}  // namespace pl
