// Back-projection onto horizontal-plane pixels, eq. (8b) / (19b), on the
// matrix cores (BF16 / FP16 modes).
//
// For one channel c, a 4x4 pixel group and 16 k_z bins the interpolation is a
// small dense product over a 16-sample window of the range grid:
//   G[kz][p] += sum_s Q_c[kz][s] B_c[s][p],
//   B_c[s][p] = K(x_p - s) exp(j k_ref l_c(p)),
// with x_p the pixel's fractional position in the window and K the 4-tap
// interpolation kernel written as a piecewise cubic (B-spline, Lagrange or
// linear).  With the real embedding A = [Re Q | Im Q] (16 kz x 32):
//   Re G = A [Re B; -Im B],   Im G = A [Im B; Re B],
// two v_mfma_f32_16x16x32_bf16 per split product; operands are BF16 hi + lo
// parts and each pair takes hi*hi + hi*lo + lo*hi (FP32 accumulation).
//
// Block = 8x8 pixel tile (four 4x4 groups, one per wavefront) x a block of up
// to 256 k_z bins sharing one reference wavenumber.  The range profiles
// arrive already split (four BF16 planes per (channel, k_z)); each channel's
// window rows are copied into LDS by direct global-to-LDS loads issued one
// channel ahead (double buffer, one barrier per channel).  A wavefront
// computes the weights of its 16 pixels for 4 channels at a time (one lane
// per pair, float64 range and carrier phase), shares them with shuffles, and
// builds its B operand in registers.
#include "device.hpp"

namespace pl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct BpmArgs {
    int n_ch, n_z, n_l, nx, ny, tiles_x, n_tiles, n_work, per_xcd, wp, rsd, kb;
    double x0, y0, dx, dy, du, inv_du, reach;
    float kc[2][4];  // K(x): |x| < 1 -> poly(kc[1], |x|); 1 <= |x| < 2 -> poly(kc[0], |x| - 1)
    double kref[kMaxBlocks];
};

__device__ __forceinline__ float kernel_eval(float x, const float (&kc)[2][4]) {
    const float ax = fabsf(x);
    const float z = ax - 1.f;
    const float y1 = ((kc[1][3] * ax + kc[1][2]) * ax + kc[1][1]) * ax + kc[1][0];
    const float y0 = ((kc[0][3] * z + kc[0][2]) * z + kc[0][1]) * z + kc[0][0];
    return ax < 1.f ? y1 : (ax < 2.f ? y0 : 0.f);
}

__device__ __forceinline__ unsigned bf16_bits(float x) {
    return static_cast<unsigned>(__builtin_bit_cast(unsigned short, static_cast<__bf16>(x)));
}
__device__ __forceinline__ float bf16_value(unsigned b) { return __uint_as_float(b << 16); }

// Split 8 values into packed BF16 hi and lo fragments (x = hi + lo).
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8& hi, bf16x8& lo) {
    u32x4 h, l;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned a = bf16_bits(v[2 * k]), b = bf16_bits(v[2 * k + 1]);
        h[k] = a | (b << 16);
        const unsigned c = bf16_bits(v[2 * k] - bf16_value(a)), d = bf16_bits(v[2 * k + 1] - bf16_value(b));
        l[k] = c | (d << 16);
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

template <int KB>
__global__ __launch_bounds__(256) void backproject_mfma_kernel(const unsigned short* __restrict__ qs,
                                                               const double* __restrict__ chan,
                                                               const double* __restrict__ llo, BpmArgs a,
                                                               float2* __restrict__ G) {
    constexpr int KT = KB / 16;  // k_z tiles of 16
    extern __shared__ unsigned smem_u[];
    int* win = reinterpret_cast<int*>(smem_u);                       // n_ch window starts (even)
    unsigned* rows = smem_u + ((a.n_ch + 63) & ~63);                  // [2][KB][rsd] dwords

    const int work = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    if (work >= a.n_work) return;  // block-uniform, before any barrier
    const int blk = work / a.n_tiles;
    const int tile = work - blk * a.n_tiles;
    const int tx0 = (tile % a.tiles_x) * 8, ty0 = (tile / a.tiles_x) * 8;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double kref_rev = a.kref[blk] * (0.5 / kPi);
    const int buf_dw = KB * a.rsd;

    // even window start of every channel for this tile
    {
        const double cx = a.x0 + (tx0 + 3.5) * a.dx, cy = a.y0 + (ty0 + 3.5) * a.dy;
        for (int c = tid; c < a.n_ch; c += 256) {
            const double* ch = chan + 4 * c;
            const double l = sqrt((cx - ch[0]) * (cx - ch[0]) + (cy - ch[1]) * (cy - ch[1])) +
                             sqrt((cx - ch[2]) * (cx - ch[2]) + (cy - ch[3]) * (cy - ch[3]));
            int s = static_cast<int>(floor((l - a.reach - llo[c]) * a.inv_du)) - 2;
            s = max(0, min(s, a.n_l - a.wp));
            win[c] = s & ~1;
        }
    }
    __syncthreads();

    // Direct global-to-LDS staging: row r of the buffer holds, for k_z bin
    // blk*KB + r, the window's 4 BF16 planes (wp samples each) = 2 wp dwords.
    // Lane t of a row copies dword t (t < 2 wp; a second pass covers t >= 64).
    const int half = a.wp / 2;
    const int t0 = lane, t1 = lane + 64;
    const unsigned lane_off0 = (t0 < 2 * a.wp) ? ((t0 / half) * a.n_l + 2 * (t0 % half)) * 2u : 0u;
    const unsigned lane_off1 = (t1 < 2 * a.wp) ? ((t1 / half) * a.n_l + 2 * (t1 % half)) * 2u : 0u;
    const bool two_pass = 2 * a.wp > 64;
    const int rows_per_wave = KB / 4;
    auto stage = [&](int c, int buf) {
        const int s0 = __builtin_amdgcn_readfirstlane(win[c]);
        for (int r = wave * rows_per_wave; r < (wave + 1) * rows_per_wave; ++r) {
            const int kz = min(blk * KB + r, a.n_z - 1);
            const char* rowg = reinterpret_cast<const char*>(
                qs + ((static_cast<size_t>(c) * a.n_z + kz) * 4) * a.n_l + s0);
            unsigned* dst = rows + buf * buf_dw + r * a.rsd;
            if (t0 < 2 * a.wp)
                __builtin_amdgcn_global_load_lds(rowg + lane_off0, dst, 4, 0, 0);
            if (two_pass && t1 < 2 * a.wp)
                __builtin_amdgcn_global_load_lds(rowg + lane_off1, dst + 64, 4, 0, 0);
        }
    };

    // this wavefront's 4x4 group and this lane's pixel in the weight batch
    const int gx = tx0 + 4 * (wave & 1), gy = ty0 + 4 * (wave >> 1);
    const int pn = lane & 15;                       // pixel of the group
    const int px = gx + (pn & 3), py = gy + (pn >> 2);
    const bool pvalid = px < a.nx && py < a.ny;
    const double xg = a.x0 + px * a.dx, yg = a.y0 + py * a.dy;
    const int kg = lane >> 4;                       // k' group of the MFMA operands

    f32x4 accr[KT], acci[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        accr[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        acci[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    stage(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // LDS dword offset of this lane's A operand: row m = lane & 15 of the
    // k_z tile, plane (Re or Im) hi, samples 8 * (kg & 1) + 0..7 of the window
    const int a_row = (lane & 15) * a.rsd;
    const int a_plane = (kg < 2 ? 0 : 2) * half + 4 * (kg & 1);

#pragma unroll 1
    for (int c0 = 0; c0 < a.n_ch; c0 += 4) {
        // weights of (pixel pn, channel c0 + lane / 16)
        float x_rel = 100.f, cr = 0.f, ci = 0.f;
        int srel = 0;
        {
            const int c = c0 + (lane >> 4);
            int i0 = 0x3fffffff;
            double u = 0.0;
            double lpath = 0.0;
            const bool ok = c < a.n_ch && pvalid;
            if (ok) {
                const double* ch = chan + 4 * c;
                lpath = sqrt((xg - ch[0]) * (xg - ch[0]) + (yg - ch[1]) * (yg - ch[1])) +
                        sqrt((xg - ch[2]) * (xg - ch[2]) + (yg - ch[3]) * (yg - ch[3]));
                u = (lpath - llo[c]) * a.inv_du;
                i0 = static_cast<int>(floor(u)) - 1;
            }
            // first tap of the group (16 lanes of the same channel)
            int m = i0;
            m = min(m, __shfl_xor(m, 1));
            m = min(m, __shfl_xor(m, 2));
            m = min(m, __shfl_xor(m, 4));
            m = min(m, __shfl_xor(m, 8));
            const int cw = win[min(c, a.n_ch - 1)];
            srel = m == 0x3fffffff ? 0 : max(0, min(m - cw, a.wp - 16)) & ~1;
            if (ok) {
                x_rel = static_cast<float>(u - static_cast<double>(cw + srel));
                const float2 car = cis_rev(kref_rev * lpath);
                cr = car.x;
                ci = car.y;
            }
        }
#pragma unroll 1
        for (int cc = 0; cc < 4; ++cc) {
            const int c = c0 + cc;
            if (c >= a.n_ch) break;
            if (c + 1 < a.n_ch) stage(c + 1, (c + 1) & 1);
            // B operand of this channel: lane (pixel n = lane & 15, k' group kg)
            const int src = cc * 16 + (lane & 15);
            const float xn = __shfl(x_rel, src), crn = __shfl(cr, src), cin = __shfl(ci, src);
            const int sr = __builtin_amdgcn_readlane(srel, cc * 16);
            const float ca = kg < 2 ? crn : -cin;   // rows of Re Q: Re B (for Re G), Im B (for Im G)
            const float cb = kg < 2 ? cin : crn;    // rows of Im Q: -Im B, Re B
            float vr[8], vi[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float kv = kernel_eval(xn - static_cast<float>(8 * (kg & 1) + t), a.kc);
                vr[t] = kv * ca;
                vi[t] = kv * cb;
            }
            bf16x8 brh, brl, bih, bil;
            split8(vr, brh, brl);
            split8(vi, bih, bil);
            // A operand rows from LDS, one k_z tile at a time
            const unsigned* abase = rows + (c & 1) * buf_dw + a_row + a_plane + sr / 2;
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                const unsigned* ap = abase + t * 16 * a.rsd;
                const u32x4 ah = u32x4{ap[0], ap[1], ap[2], ap[3]};
                const u32x4 al = u32x4{ap[half + 0], ap[half + 1], ap[half + 2], ap[half + 3]};
                const bf16x8 vah = __builtin_bit_cast(bf16x8, ah), val = __builtin_bit_cast(bf16x8, al);
                accr[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, brh, accr[t], 0, 0, 0);
                acci[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, bih, acci[t], 0, 0, 0);
                accr[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, brl, accr[t], 0, 0, 0);
                acci[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, bil, acci[t], 0, 0, 0);
                accr[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(val, brh, accr[t], 0, 0, 0);
                acci[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(val, bih, acci[t], 0, 0, 0);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
    }

    // D layout: lane holds column (pixel) lane & 15, rows 4 * (lane >> 4) + v
    if (pvalid) {
        float2* out = G + (static_cast<size_t>(py) * a.nx + px) * a.n_z;
#pragma unroll
        for (int t = 0; t < KT; ++t) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kz = blk * KB + 16 * t + 4 * kg + v;
                if (kz < a.n_z) out[kz] = make_float2(accr[t][v], acci[t][v]);
            }
        }
    }
}

template <int KB>
int launch_kb(const BpmArgs& a, size_t smem, unsigned blocks, hipStream_t s, const unsigned short* qs,
              const double* chan, const double* llo, float2* G) {
    auto fn = backproject_mfma_kernel<KB>;
    if (smem > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem));
        if (e != hipSuccess) return fail(PL_EDEVICE, "MFMA back-projection LDS of %zu bytes: %s", smem, hipGetErrorString(e));
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), smem, s, qs, chan, llo, a, G);
    return check_launch("back-projection (MFMA)");
}

}  // namespace

int launch_backproject_mfma(const HybridPlan& p, const DeviceTables& dt, const unsigned short* qs, char* ws,
                            float2* G, hipStream_t s) {
    BpmArgs a{};
    a.n_ch = p.n_ch;
    a.n_z = p.n_z;
    a.n_l = p.n_l;
    a.nx = p.nx;
    a.ny = p.ny;
    a.tiles_x = p.tiles_x;
    a.n_tiles = p.tiles_x * p.tiles_y;
    a.n_work = a.n_tiles * p.n_blocks;
    a.per_xcd = (a.n_work + 7) / 8;
    a.wp = p.window;
    a.rsd = p.window_pad;
    a.kb = p.block;
    a.x0 = p.x0;
    a.y0 = p.y0;
    a.dx = p.dx;
    a.dy = p.dy;
    a.du = p.du;
    a.inv_du = 1.0 / p.du;
    a.reach = std::hypot(7.0 * p.dx, 7.0 * p.dy);
    for (int j = 0; j < 4; ++j) {
        a.kc[0][j] = p.coef[0][j];
        a.kc[1][j] = p.coef[1][j];
    }
    for (int b = 0; b < kMaxBlocks; ++b) a.kref[b] = p.kref[b];
    if (p.window < 16 || p.window > 64 || (p.window & 1) || p.window > p.n_l || p.window_pad != 2 * p.window + 1)
        return fail(PL_EUNSUPPORTED, "MFMA back-projection window %d out of range", p.window);
    const size_t smem = static_cast<size_t>((p.n_ch + 63) & ~63) * 4 + 2ull * p.block * p.window_pad * 4;
    if (smem > kMaxLds) return fail(PL_EUNSUPPORTED, "MFMA back-projection needs %zu bytes of LDS", smem);
    const unsigned blocks = static_cast<unsigned>(8 * a.per_xcd);
    const double* llo = reinterpret_cast<const double*>(ws + p.off_llo);
    switch (p.block) {
        case 64: return launch_kb<64>(a, smem, blocks, s, qs, dt.chan, llo, G);
        case 128: return launch_kb<128>(a, smem, blocks, s, qs, dt.chan, llo, G);
        case 192: return launch_kb<192>(a, smem, blocks, s, qs, dt.chan, llo, G);
        case 256: return launch_kb<256>(a, smem, blocks, s, qs, dt.chan, llo, G);
        default: return fail(PL_EUNSUPPORTED, "MFMA back-projection block of %d k_z bins", p.block);
    }
}

}  // namespace pl
