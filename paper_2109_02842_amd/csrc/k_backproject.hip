// Interpolated back-projection onto horizontal-plane pixels, eq. (8b) / (19b):
//   G[p][kz] = sum_c exp(j k_ref(block(kz)) l_c(p)) * I(q_{c,kz}, u_c(p)),
//   u_c(p) = (l_c(p) - l_lo[c]) / du,  l_c(p) = rho_T + rho_R,
// with I a 4-tap interpolation (cubic B-spline on prefiltered samples,
// cubic Lagrange, or linear).
//
// Mapping on gfx950: one block = one pixel tile x one block of 64 k_z bins;
// lane = k_z bin, so the interpolation weights and the carrier of a
// (pixel, channel) pair are wavefront-uniform.  They are computed once per
// pair (range in float64, carrier phase range-reduced in float64) by one
// lane each and broadcast with readlane; every k_z bin then costs four LDS
// reads and twelve FMAs.  The channel's range window for the tile is staged
// in LDS (double-buffered: the next channel's rows are loaded into registers
// while the current one is consumed).  Blocks are assigned so that each XCD
// works on a contiguous range of (k_z block, tile) work items, which keeps
// the range profiles it reads in its own L2.
#include "device.hpp"

namespace pl {
namespace {

struct BpjArgs {
    int n_ch, n_z, n_l, nx, ny, tiles_x, n_tiles, n_work, per_xcd, window, wpad, pad_;
    double x0, y0, dx, dy, du, inv_du, reach;
    float coef[4][4];
    double kref[kMaxBlocks];
};

__device__ __forceinline__ float rdl(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <int TX, int TY, int E>
__global__ __launch_bounds__(256) void backproject_kernel(const float2* __restrict__ q,
                                                          const double* __restrict__ chan,
                                                          const double* __restrict__ llo, BpjArgs a,
                                                          float2* __restrict__ G) {
    constexpr int PPW = TX * TY / 4;  // pixels per wavefront
    constexpr int CPB = 64 / PPW;     // channels per weight batch
    static_assert(PPW * CPB == 64, "tile must give 1, 4 or 16 pixels per wavefront");
    extern __shared__ int smem_i[];
    int* win = smem_i;                                                            // n_ch window starts
    float2* qbuf = reinterpret_cast<float2*>(smem_i + ((a.n_ch + 63) & ~63));     // [2][64][wpad]

    const int work = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    if (work >= a.n_work) return;  // block-uniform, before any barrier
    const int blk = work / a.n_tiles;
    const int tile = work - blk * a.n_tiles;
    const int tx0 = (tile % a.tiles_x) * TX, ty0 = (tile / a.tiles_x) * TY;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int kap = blk * 64 + lane;
    const double kref_rev = a.kref[blk] * (0.5 / kPi);
    const int buf_stride = 64 * a.wpad;

    // window start of every channel for this tile
    {
        const double cx = a.x0 + (tx0 + 0.5 * (TX - 1)) * a.dx;
        const double cy = a.y0 + (ty0 + 0.5 * (TY - 1)) * a.dy;
        for (int c = tid; c < a.n_ch; c += 256) {
            const double* ch = chan + 4 * c;
            const double l = hypot(cx - ch[0], cy - ch[1]) + hypot(cx - ch[2], cy - ch[3]);
            int s = static_cast<int>(floor((l - a.reach - llo[c]) * a.inv_du)) - 1;
            s = max(0, min(s, a.n_l - a.window));
            win[c] = s;
        }
    }
    __syncthreads();

    // staging: wavefront w moves rows kz_local in [16w, 16w + 16)
    float2 stage[16][E];
    auto load_rows = [&](int c) {
        const int s0 = win[c];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int kl = wave * 16 + r;
            const int kz = blk * 64 + kl;
            const float2* src = q + (static_cast<size_t>(c) * a.n_z + kz) * a.n_l + s0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int i = lane + 64 * e;
                stage[r][e] = (kz < a.n_z && i < a.window) ? src[i] : make_float2(0.f, 0.f);
            }
        }
    };
    auto store_rows = [&](int buf) {
        float2* dst = qbuf + buf * buf_stride;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int kl = wave * 16 + r;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int i = lane + 64 * e;
                if (i < a.window) dst[kl * a.wpad + i] = stage[r][e];
            }
        }
    };

    float2 acc[PPW];
#pragma unroll
    for (int j = 0; j < PPW; ++j) acc[j] = make_float2(0.f, 0.f);

    load_rows(0);
    store_rows(0);
    __syncthreads();

    // this lane's pixel in the weight batches
    const int pj = lane % PPW;
    const int pl = wave * PPW + pj;
    const int px = tx0 + pl % TX, py = ty0 + pl / TX;
    const bool pvalid = px < a.nx && py < a.ny;
    const double xg = a.x0 + px * a.dx, yg = a.y0 + py * a.dy;

    for (int c0 = 0; c0 < a.n_ch; c0 += CPB) {
        // weights of (pixel pj, channel c0 + lane / PPW)
        int my_i0 = 0;
        float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f, cr = 0.f, ci = 0.f;
        {
            const int c = c0 + lane / PPW;
            if (c < a.n_ch && pvalid) {
                const double* ch = chan + 4 * c;
                const double l = hypot(xg - ch[0], yg - ch[1]) + hypot(xg - ch[2], yg - ch[3]);
                const double u = (l - llo[c]) * a.inv_du;
                const double fl = floor(u);
                const float t = static_cast<float>(u - fl);
                my_i0 = static_cast<int>(fl) - 1 - win[c];
                my_i0 = max(0, min(my_i0, a.window - 4));
                w0 = ((a.coef[0][3] * t + a.coef[0][2]) * t + a.coef[0][1]) * t + a.coef[0][0];
                w1 = ((a.coef[1][3] * t + a.coef[1][2]) * t + a.coef[1][1]) * t + a.coef[1][0];
                w2 = ((a.coef[2][3] * t + a.coef[2][2]) * t + a.coef[2][1]) * t + a.coef[2][0];
                w3 = ((a.coef[3][3] * t + a.coef[3][2]) * t + a.coef[3][1]) * t + a.coef[3][0];
                const float2 car = cis_rev(kref_rev * l);
                cr = car.x;
                ci = car.y;
            }
        }
        for (int cc = 0; cc < CPB; ++cc) {
            const int c = c0 + cc;
            if (c >= a.n_ch) break;
            const bool more = c + 1 < a.n_ch;
            if (more) load_rows(c + 1);
            const float2* base = qbuf + (c & 1) * buf_stride + lane * a.wpad;
#pragma unroll
            for (int j = 0; j < PPW; ++j) {
                const int L = cc * PPW + j;
                const int i0 = __builtin_amdgcn_readlane(my_i0, L);
                const float v0 = rdl(w0, L), v1 = rdl(w1, L), v2 = rdl(w2, L), v3 = rdl(w3, L);
                const float kr = rdl(cr, L), ki = rdl(ci, L);
                const float2 q0 = base[i0], q1 = base[i0 + 1], q2 = base[i0 + 2], q3 = base[i0 + 3];
                const float re = v0 * q0.x + v1 * q1.x + v2 * q2.x + v3 * q3.x;
                const float im = v0 * q0.y + v1 * q1.y + v2 * q2.y + v3 * q3.y;
                acc[j].x += kr * re - ki * im;
                acc[j].y += kr * im + ki * re;
            }
            if (more) store_rows((c + 1) & 1);
            __syncthreads();
        }
    }

    if (kap < a.n_z) {
#pragma unroll
        for (int j = 0; j < PPW; ++j) {
            const int l = wave * PPW + j;
            const int x = tx0 + l % TX, y = ty0 + l / TX;
            if (x < a.nx && y < a.ny) G[(static_cast<size_t>(y) * a.nx + x) * a.n_z + kap] = acc[j];
        }
    }
}

template <int TX, int TY, int E>
int launch_tile(const BpjArgs& a, size_t smem, unsigned blocks, hipStream_t s, const float2* q,
                const double* chan, const double* llo, float2* G) {
    auto fn = backproject_kernel<TX, TY, E>;
    if (smem > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(smem));
        if (e != hipSuccess) return fail(PL_EDEVICE, "back-projection LDS of %zu bytes: %s", smem, hipGetErrorString(e));
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), smem, s, q, chan, llo, a, G);
    return check_launch("back-projection");
}

}  // namespace

int launch_backproject(const HybridPlan& p, const DeviceTables& dt, const float2* q, char* ws, float2* G,
                       hipStream_t s) {
    BpjArgs a{};
    a.n_ch = p.n_ch;
    a.n_z = p.n_z;
    a.n_l = p.n_l;
    a.nx = p.nx;
    a.ny = p.ny;
    a.tiles_x = p.tiles_x;
    a.n_tiles = p.tiles_x * p.tiles_y;
    a.n_work = a.n_tiles * p.n_blocks;
    a.per_xcd = (a.n_work + 7) / 8;
    a.window = p.window;
    a.wpad = p.window_pad;
    a.x0 = p.x0;
    a.y0 = p.y0;
    a.dx = p.dx;
    a.dy = p.dy;
    a.du = p.du;
    a.inv_du = 1.0 / p.du;
    a.reach = std::hypot((p.tile_x - 1) * p.dx, (p.tile_y - 1) * p.dy);  // 2 x half-diagonal
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 4; ++j) a.coef[k][j] = p.coef[k][j];
    for (int b = 0; b < kMaxBlocks; ++b) a.kref[b] = p.kref[b];
    if (p.window < 4 || p.window > 128 || p.window > p.n_l)
        return fail(PL_EUNSUPPORTED, "back-projection window %d out of range", p.window);
    const size_t smem = static_cast<size_t>((p.n_ch + 63) & ~63) * 4 + 2ull * 64 * p.window_pad * 8;
    if (smem > 160 * 1024) return fail(PL_EUNSUPPORTED, "back-projection needs %zu bytes of LDS", smem);
    const unsigned blocks = static_cast<unsigned>(8 * a.per_xcd);
    const double* llo = reinterpret_cast<const double*>(ws + p.off_llo);
    const bool two = p.window > 64;
    if (p.tile_x == 8 && p.tile_y == 8)
        return two ? launch_tile<8, 8, 2>(a, smem, blocks, s, q, dt.chan, llo, G)
                   : launch_tile<8, 8, 1>(a, smem, blocks, s, q, dt.chan, llo, G);
    if (p.tile_x == 4 && p.tile_y == 4)
        return two ? launch_tile<4, 4, 2>(a, smem, blocks, s, q, dt.chan, llo, G)
                   : launch_tile<4, 4, 1>(a, smem, blocks, s, q, dt.chan, llo, G);
    if (p.tile_x == 2 && p.tile_y == 2)
        return two ? launch_tile<2, 2, 2>(a, smem, blocks, s, q, dt.chan, llo, G)
                   : launch_tile<2, 2, 1>(a, smem, blocks, s, q, dt.chan, llo, G);
    return fail(PL_EUNSUPPORTED, "no back-projection kernel for a %dx%d tile", p.tile_x, p.tile_y);
}

}  // namespace pl
