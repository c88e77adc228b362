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
// in LDS, double-buffered: the next channel's rows are copied into the other
// buffer before the current one is consumed (the other resident waves hide
// the load latency), one barrier per channel.  Blocks are assigned so that each XCD
// works on a contiguous range of (k_z block, tile) work items, which keeps
// the range profiles it reads in its own L2.
#include <cstring>

#include "device.hpp"

namespace pl {
namespace {

struct BpjArgs {
    int n_ch, n_z, n_l, nx, ny, tiles_x, n_tiles, n_work, per_xcd, window, wpad, rows;
    double x0, y0, dx, dy, du, inv_du, reach;
    float coef[4][4];
    double kref[kMaxBlocks];
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
// gfx9 raw-buffer descriptor word 3: 32-bit data format, no swizzle
constexpr int kBufferFlags = 0x00020000;

// Buffer descriptor of a wavefront-uniform slab.  The address halves go
// through readfirstlane so the compiler knows the descriptor is uniform and
// emits plain scalar-descriptor loads (no waterfall loops).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const float2* p, unsigned bytes) {
    const unsigned long long a = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
    void* u = reinterpret_cast<void*>((static_cast<unsigned long long>(hi) << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(u, 0, __builtin_amdgcn_readfirstlane(bytes), kBufferFlags);
}

__device__ __forceinline__ float2 load_c64(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, __builtin_amdgcn_readfirstlane(soff), 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}


// TX x TY pixel tile, KPL k_z bins per lane (a block of 64 * KPL bins shares
// one reference wavenumber), NW wavefronts per block, OCC the wavefronts per
// SIMD the LDS footprint allows (it caps the registers at 512 / OCC).
// KZREF: every k_z bin has its own reference krz[kz] (the paper's k_rho0 of
// eq. 8b/19b), so each lane forms its carrier per (pixel, channel) from the
// broadcast float64 range, range-reduced in float64.
template <int TX, int TY, int KPL, int NW, int OCC, bool KZREF>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC))) void backproject_kernel(const float2* __restrict__ q,
                                                              const double* __restrict__ chan,
                                                              const double* __restrict__ llo,
                                                              const double* __restrict__ krz, BpjArgs a,
                                                              float2* __restrict__ G) {
    constexpr int NT = 64 * NW;
    constexpr int PPW = TX * TY / NW;   // pixels per wavefront
    constexpr int CPB = 64 / PPW;       // channels per weight batch
    constexpr int ROWS = 64 * KPL;      // k_z rows staged per channel
    constexpr int RPW = ROWS / NW;      // rows staged by each wavefront
    constexpr int PASS = RPW < 16 ? RPW : 16;
    static_assert(PPW * CPB == 64, "a weight batch must fill the wavefront");
    static_assert(RPW % PASS == 0, "rows per wavefront");
    extern __shared__ int smem_i[];
    int* win = smem_i;                                                            // n_ch window starts
    float2* qbuf = reinterpret_cast<float2*>(smem_i + ((a.n_ch + 63) & ~63));     // [2][ROWS][wpad]

    const int work = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    if (work >= a.n_work) return;  // block-uniform, before any barrier
    const int blk = work / a.n_tiles;
    const int tile = work - blk * a.n_tiles;
    const int tx0 = (tile % a.tiles_x) * TX, ty0 = (tile / a.tiles_x) * TY;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront-uniform
    const double kref_rev = a.kref[blk] * (0.5 / kPi);
    double krz_rev[KPL];
#pragma unroll
    for (int r = 0; r < KPL; ++r)
        krz_rev[r] = KZREF ? krz[min(blk * ROWS + (tid & 63) + 64 * r, a.n_z - 1)] * (0.5 / kPi) : 0.0;
    const int buf_stride = ROWS * a.wpad;

    // window start of every channel for this tile
    {
        const double cx = a.x0 + (tx0 + 0.5 * (TX - 1)) * a.dx;
        const double cy = a.y0 + (ty0 + 0.5 * (TY - 1)) * a.dy;
        for (int c = tid; c < a.n_ch; c += NT) {
            const double* ch = chan + 4 * c;
            const double l = sqrt((cx - ch[0]) * (cx - ch[0]) + (cy - ch[1]) * (cy - ch[1])) +
                             sqrt((cx - ch[2]) * (cx - ch[2]) + (cy - ch[3]) * (cy - ch[3]));
            int s = static_cast<int>(floor((l - a.reach - llo[c]) * a.inv_du)) - 1;
            s = max(0, min(s, a.n_l - a.window));
            win[c] = s;
        }
    }
    __syncthreads();

    // Staging: wavefront w copies rows [w * RPW, (w + 1) * RPW) of the k_z
    // block.  Every load stays in bounds: rows past the last k_z bin repeat it
    // and lanes past the window repeat its last sample; only the LDS stores
    // are predicated (repeated rows feed lanes whose results are dropped).
    const int kz_first = blk * ROWS + wave * RPW;
    const int ie0 = min(lane, a.window - 1);
    const int ie1 = min(lane + 64, a.window - 1);
    // Rows are read with buffer loads: a uniform descriptor for the channel's
    // slab q[c][:][:], a 32-bit lane offset and a scalar row offset, so no
    // per-lane 64-bit addresses are kept live.
    float2 stage[PASS];
    const unsigned slab_bytes = static_cast<unsigned>(a.n_z) * a.n_l * 8u;
    const unsigned row_bytes = static_cast<unsigned>(a.n_l) * 8u;
#define PL_STAGE(C_, BUF_)                                                                    \
    {                                                                                         \
        const int s0_ = __builtin_amdgcn_readfirstlane(win[C_]);                              \
        const __amdgpu_buffer_rsrc_t rs_ =                                                    \
            slab_rsrc(q + static_cast<size_t>(C_) * a.n_z * a.n_l, slab_bytes);               \
        const unsigned v0_ = static_cast<unsigned>(s0_ + ie0) * 8u;                           \
        const unsigned v1_ = static_cast<unsigned>(s0_ + ie1) * 8u;                           \
        float2* dst_ = qbuf + (BUF_) * buf_stride + wave * RPW * a.wpad;                      \
        _Pragma("unroll") for (int r0 = 0; r0 < RPW; r0 += PASS) {                            \
            _Pragma("unroll") for (int r = 0; r < PASS; ++r) {                                \
                const unsigned so_ = static_cast<unsigned>(min(kz_first + r0 + r, a.n_z - 1)) * row_bytes; \
                stage[r] = load_c64(rs_, v0_, so_);                                           \
            }                                                                                 \
            _Pragma("unroll") for (int r = 0; r < PASS; ++r)                                  \
                if (lane < a.window) dst_[(r0 + r) * a.wpad + lane] = stage[r];               \
            if (a.window > 64) {                                                              \
                _Pragma("unroll") for (int r = 0; r < PASS; ++r) {                            \
                    const unsigned so_ = static_cast<unsigned>(min(kz_first + r0 + r, a.n_z - 1)) * row_bytes; \
                    stage[r] = load_c64(rs_, v1_, so_);                                       \
                }                                                                             \
                _Pragma("unroll") for (int r = 0; r < PASS; ++r)                              \
                    if (lane + 64 < a.window) dst_[(r0 + r) * a.wpad + lane + 64] = stage[r]; \
            }                                                                                 \
        }                                                                                     \
    }

    float2 acc[PPW][KPL];
#pragma unroll
    for (int j = 0; j < PPW; ++j)
#pragma unroll
        for (int r = 0; r < KPL; ++r) acc[j][r] = make_float2(0.f, 0.f);

    PL_STAGE(0, 0)
    __syncthreads();

    // this lane's pixel in the weight batches
    const int pj = lane % PPW;
    const int pl = wave * PPW + pj;
    const int px = tx0 + pl % TX, py = ty0 + pl / TX;
    const bool pvalid = px < a.nx && py < a.ny;
    const double xg = a.x0 + px * a.dx, yg = a.y0 + py * a.dy;

#pragma unroll 1
    for (int c0 = 0; c0 < a.n_ch; c0 += CPB) {
        // weights of (pixel pj, channel c0 + lane / PPW): range in float64,
        // taps and cubic weights, carrier exp(j k_ref l) with float64 phase
        int my_i0 = 0;
        float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f, cr = 0.f, ci = 0.f;
        double my_l = 0.0;
        {
            const int c = c0 + lane / PPW;
            if (c < a.n_ch && pvalid) {
                const double* ch = chan + 4 * c;
                const double l = sqrt((xg - ch[0]) * (xg - ch[0]) + (yg - ch[1]) * (yg - ch[1])) +
                                 sqrt((xg - ch[2]) * (xg - ch[2]) + (yg - ch[3]) * (yg - ch[3]));
                const double u = (l - llo[c]) * a.inv_du;
                const double fl = floor(u);
                const float t = static_cast<float>(u - fl);
                my_i0 = static_cast<int>(fl) - 1 - win[c];
                my_i0 = max(0, min(my_i0, a.window - 4));
                w0 = ((a.coef[0][3] * t + a.coef[0][2]) * t + a.coef[0][1]) * t + a.coef[0][0];
                w1 = ((a.coef[1][3] * t + a.coef[1][2]) * t + a.coef[1][1]) * t + a.coef[1][0];
                w2 = ((a.coef[2][3] * t + a.coef[2][2]) * t + a.coef[2][1]) * t + a.coef[2][0];
                w3 = ((a.coef[3][3] * t + a.coef[3][2]) * t + a.coef[3][1]) * t + a.coef[3][0];
                if (KZREF) {
                    my_l = l;
                } else {
                    const float2 car = cis_rev(kref_rev * l);
                    cr = car.x;
                    ci = car.y;
                }
            }
        }
#pragma unroll 1
        for (int cc = 0; cc < CPB; ++cc) {
            const int c = c0 + cc;
            if (c >= a.n_ch) break;
            if (c + 1 < a.n_ch) PL_STAGE(c + 1, (c + 1) & 1)
            const float2* base = qbuf + (c & 1) * buf_stride + lane * a.wpad;
#pragma unroll
            for (int j = 0; j < PPW; ++j) {
                const int L = cc * PPW + j;
                const int i0 = __builtin_amdgcn_readlane(my_i0, L);
                const float v0 = rdl(w0, L), v1 = rdl(w1, L), v2 = rdl(w2, L), v3 = rdl(w3, L);
                float kr = rdl(cr, L), ki = rdl(ci, L);
                double lb = 0.0;
                if (KZREF) {
                    const long long bits = __double_as_longlong(my_l);
                    const int lo = __builtin_amdgcn_readlane(static_cast<int>(bits), L);
                    const int hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), L);
                    lb = __hiloint2double(hi, lo);
                }
                const float2* b = base + i0;
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    if (KZREF) {
                        const float2 car = cis_rev(krz_rev[r] * lb);
                        kr = car.x;
                        ki = car.y;
                    }
                    const float2* br = b + r * 64 * a.wpad;
                    const float2 q0 = br[0], q1 = br[1], q2 = br[2], q3 = br[3];
                    const float re = v0 * q0.x + v1 * q1.x + v2 * q2.x + v3 * q3.x;
                    const float im = v0 * q0.y + v1 * q1.y + v2 * q2.y + v3 * q3.y;
                    acc[j][r].x = fmaf(kr, re, acc[j][r].x);
                    acc[j][r].x = fmaf(-ki, im, acc[j][r].x);
                    acc[j][r].y = fmaf(kr, im, acc[j][r].y);
                    acc[j][r].y = fmaf(ki, re, acc[j][r].y);
                }
            }
            __syncthreads();
        }
    }
#undef PL_STAGE

#pragma unroll
    for (int j = 0; j < PPW; ++j) {
        const int l = wave * PPW + j;
        const int x = tx0 + l % TX, y = ty0 + l / TX;
        if (x < a.nx && y < a.ny) {
#pragma unroll
            for (int r = 0; r < KPL; ++r) {
                const int kz = blk * ROWS + lane + 64 * r;
                if (kz < a.n_z) G[(static_cast<size_t>(y) * a.nx + x) * a.n_z + kz] = acc[j][r];
            }
        }
    }
}

template <int TX, int TY, int KPL, int NW, int OCC, bool KZREF = false>
int launch_variant(const BpjArgs& a, size_t smem, unsigned blocks, hipStream_t s, const float2* q,
                   const double* chan, const double* llo, const double* krz, float2* G) {
    auto fn = backproject_kernel<TX, TY, KPL, NW, OCC, KZREF>;
    if (smem > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(smem));
        if (e != hipSuccess) return fail(PL_EDEVICE, "back-projection LDS of %zu bytes: %s", smem, hipGetErrorString(e));
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * NW), smem, s, q, chan, llo, krz, a, G);
    return check_launch("back-projection");
}


// ---------------------------------------------------------------------------
// Pixel-per-lane variant (the default): one workgroup = one 8x8 pixel tile x
// KB k_z bins; lane = pixel, wavefront w owns k_z rows [RW w, RW (w + 1)).
// The weights and carrier of a (pixel, channel) pair are computed once per
// workgroup (wavefront w for the w-th channel of a batch of 4, at the start
// of the batch) and shared through LDS, so nothing is broadcast per pixel.  A
// pixel reads its four tap samples with four ds_read_b64 (32 bytes of LDS
// and twelve FMAs per (pixel, k_z) term).  The reads are kept apart by an
// empty asm with a memory clobber: the compiler would pair adjacent ones
// into ds_read2_b64, which serves fewer lanes per cycle on gfx950 (paired,
// this form ran slower than two aligned 16-byte reads of five samples with
// a zero weight; unpaired it is 9 % faster).  The channel's window rows (even start)
// are copied into LDS by 16-byte direct global-to-LDS loads one channel
// ahead, double-buffered.  The kernel is bound by instruction issue with
// its latencies covered by other workgroups: LDS per workgroup (8 KiB of
// weight slots and the two row buffers) is what sets how many fit a CU.
struct BpgArgs {
    int n_ch, n_z, n_l, nx, ny, tiles_x, n_tiles, n_work, per_xcd, nchk, mono;
    double x0, y0, dx, dy, inv_du, reach;
    float coef[4][4];
    double kref[kMaxBlocks];
};

// GatherTileEntry (internal.hpp): the per (tile, channel) geometry table.


// One scan of a batch: its arguments and byte offsets of its range profiles,
// tile table and spectrum in the batch workspace.
struct BatchScanDesc {
    BpgArgs a;
    unsigned long long q_off, tab_off, g_off;
};

constexpr int kGatherWaves = 4;   // wavefronts per workgroup
constexpr int kGatherBatch = 4;   // channels per weight batch

typedef __attribute__((address_space(3))) unsigned char* lds_bytes_t;
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) GatherTileEntry* const_tile_t;
typedef const __attribute__((address_space(4))) float2* const_f2_t;
#define PL_LDS_COPY16(RS, DST, VOFF) __builtin_amdgcn_raw_ptr_buffer_load_lds((RS), (DST), 16, (VOFF), 0, 0, 0)
#else
// host pass: parsed only, never run (the builtin is device-only)
typedef const GatherTileEntry* const_tile_t;
typedef const float2* const_f2_t;
#define PL_LDS_COPY16(RS, DST, VOFF) ((void)(RS), (void)(DST), (void)(VOFF))
#endif

// RSC 16-byte chunks per LDS row, of which nchk (the window) are staged.
// With A, B = (l_c -+ reach - l_lo) / du for the tile centre's range l_c,
// every pixel has u in [A, B]; the window starts at s in
// [floor(A) - 3, floor(A) - 2] (even), so a first tap f = floor(u) - 1 has
// f - s in [1, ceil(B - A) + 2], at most the window length minus 6 (the
// planner's window is ceil(2 reach / du) + 8 samples or more: the bound
// plus one sample against float rounding).  A pixel reads the samples
// [f - s, f - s + 4), inside the window while f - s <= wpl - 4.
// One (k_z block, tile) work item; tab = the scan's tile table; smem = the
// workgroup's LDS (the weight slots, then the two row buffers).
//
// A channel's rows are copied into LDS by buffer loads that write LDS
// directly: the descriptor's base is the channel's window start and its
// size the rest of the channel, both scalar, so the copies take no vector
// instructions; lanes whose chunk lies past the window (row padding that no
// pixel reads) get an offset beyond the descriptor's size.  The batch of
// NB channels is unrolled, so which buffer a channel uses is a constant.
template <int KB, int RSC>
__device__ __forceinline__ void gather_tile(const BpgArgs& a, const float2* __restrict__ q,
                                            const GatherTileEntry* __restrict__ tab, float2* __restrict__ G,
                                            int blk, int tile, unsigned char* smem) {
    constexpr int NW = kGatherWaves, RW = KB / NW, NB = kGatherBatch;
    constexpr int NIW = (KB * RSC + 64 * NW - 1) / (64 * NW);  // copy instructions per wavefront
    constexpr unsigned kBufBytes = KB * RSC * 16;
    static_assert((KB * RSC) % 64 == 0, "every copy instruction fills 64 whole chunks");
    static_assert(NB % 2 == 0, "a batch starts on the first row buffer");
    float4* wts = reinterpret_cast<float4*>(smem);   // [NB][2][64]
    constexpr unsigned lds_q = NB * 2 * 64 * 16;

    const int tx0 = (tile % a.tiles_x) * 8, ty0 = (tile / a.tiles_x) * 8;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wpl = 2 * a.nchk;
    const float kref_rev_f = static_cast<float>(a.kref[blk] * (0.5 / kPi));
    const float inv_du_f = static_cast<float>(a.inv_du);
    const GatherTileEntry* tt = tab + static_cast<size_t>(tile) * a.n_ch;
    const float2* tc = reinterpret_cast<const float2*>(tab + static_cast<size_t>(a.n_tiles) * a.n_ch) +
                       (static_cast<size_t>(blk) * a.n_tiles + tile) * a.n_ch;
    // wavefront-uniform and immutable during the launch: read through the
    // constant address space (scalar loads)
    const const_tile_t ttc = reinterpret_cast<const_tile_t>(reinterpret_cast<unsigned long long>(tt));
    const const_f2_t tcc = reinterpret_cast<const_f2_t>(reinterpret_cast<unsigned long long>(tc));

    // copy offsets (bytes from the channel's window start); 0x80000000 is
    // beyond any descriptor size (a channel's profiles are under 2 GiB)
    unsigned doff[NIW];
#pragma unroll
    for (int j = 0; j < NIW; ++j) {
        const int g = (wave + NW * j) * 64 + lane;
        const int r = g / RSC, k = g - r * RSC;
        const int kz = min(blk * KB + r, a.n_z - 1);
        doff[j] = (r < KB && k < a.nchk) ? static_cast<unsigned>((kz * a.n_l + 2 * k) * 8) : 0x80000000u;
    }
    const size_t chan_elems = static_cast<size_t>(a.n_z) * a.n_l;
    const unsigned chan_bytes = static_cast<unsigned>(chan_elems * 8);
    auto stage = [&](int c, int buf, int win) {
        const __amdgpu_buffer_rsrc_t rs = slab_rsrc(q + c * chan_elems + win, chan_bytes - 8u * win);
        const lds_bytes_t dst = (lds_bytes_t)(smem + lds_q + buf * kBufBytes);  // generic to LDS address
#pragma unroll
        for (int j = 0; j < NIW; ++j) {
            const int i = wave + NW * j;
            if (i * 64 < KB * RSC) PL_LDS_COPY16(rs, dst + i * 1024, doff[j]);
        }
    };

    // this lane's pixel and its offset from the tile centre
    const int px = tx0 + (lane & 7), py = ty0 + (lane >> 3);
    const bool pvalid = px < a.nx && py < a.ny;
    const float ox = ((lane & 7) - 3.5f) * static_cast<float>(a.dx), oy = ((lane >> 3) - 3.5f) * static_cast<float>(a.dy);
    const float oo = ox * ox + oy * oy;

    // weights of (this lane's pixel, channel c) into slot [wave]: four tap
    // weights, carrier, byte offset of the first tap in the row.  Lanes of
    // pixels outside the image compute them like the others (their offset
    // is clamped into the row; their sums are never written); a channel past
    // the last one is never read.
    auto weights = [&](int c) {
        const int ce = min(c, a.n_ch - 1);
        const GatherTileEntry e = ttc[ce];
        // range offset from the tile centre (see GatherTileEntry)
        const float sT = 2.f * (e.xt * ox + e.yt * oy) + oo;
        float dl = sT * __builtin_amdgcn_rcpf(e.dt + __builtin_amdgcn_sqrtf(e.dt * e.dt + sT));
        if (a.mono) {
            dl += dl;
        } else {
            const float sR = 2.f * (e.xr * ox + e.yr * oy) + oo;
            dl += sR * __builtin_amdgcn_rcpf(e.dr + __builtin_amdgcn_sqrtf(e.dr * e.dr + sR));
        }
        const float uu = e.uf + dl * inv_du_f;
        const float fv = floorf(uu);
        const float t = uu - fv;
        // within the window by the bound above; the clamp keeps every read
        // inside the staged row whatever the rounding
        const int i0 = max(0, min(e.base + static_cast<int>(fv), wpl - 4));
        float w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            w[j] = ((a.coef[j][3] * t + a.coef[j][2]) * t + a.coef[j][1]) * t + a.coef[j][0];
        // carrier exp(j k_ref l): the centre's (tile table) times the offset's
        const float2 c0 = tcc[ce];
        const float2 c1 = cis_rev_f(kref_rev_f * dl);   // |dl| spans a tile: a few revolutions
        float4* slot = wts + wave * 2 * 64 + lane;
        slot[0] = make_float4(w[0], w[1], w[2], w[3]);
        slot[64] = make_float4(c0.x * c1.x - c0.y * c1.y, c0.x * c1.y + c0.y * c1.x, __int_as_float(i0 * 8), 0.f);
    };

    float2 acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = make_float2(0.f, 0.f);

    __syncthreads();  // LDS free (the batch kernel reuses it per item)
    stage(0, 0, ttc[0].win);

    const unsigned row0 = static_cast<unsigned>(wave * RW * RSC * 16);
#pragma unroll 1
    for (int c0 = 0; c0 < a.n_ch; c0 += NB) {
        // window starts of the channels staged during this batch (scalar
        // loads, issued together)
        int wn[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) wn[k] = ttc[min(c0 + 1 + k, a.n_ch - 1)].win;
        // the previous batch's slots are read (barrier at the end of its
        // last channel), so this batch's weights can take them
        weights(c0 + wave);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) {
            const int c = c0 + cc;
            if (c >= a.n_ch) break;
            if (c + 1 < a.n_ch) stage(c + 1, (cc + 1) & 1, wn[cc]);
            const float4* slot = wts + cc * 2 * 64 + lane;
            const float4 wa = slot[0], wb = slot[64];
            const unsigned off = __float_as_uint(wb.z);
            const unsigned char* rp = smem + lds_q + (cc & 1) * kBufBytes + row0 + off;
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const float2* cp = reinterpret_cast<const float2*>(rp + r * RSC * 16);
                // four separate 8-byte reads: the empty asm keeps the
                // compiler from pairing them into ds_read2_b64
                float2 q[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    q[j] = cp[j];
                    asm volatile("" ::: "memory");
                }
                const float re = wa.x * q[0].x + wa.y * q[1].x + wa.z * q[2].x + wa.w * q[3].x;
                const float im = wa.x * q[0].y + wa.y * q[1].y + wa.z * q[2].y + wa.w * q[3].y;
                acc[r].x = fmaf(wb.x, re, acc[r].x);
                acc[r].x = fmaf(-wb.y, im, acc[r].x);
                acc[r].y = fmaf(wb.x, im, acc[r].y);
                acc[r].y = fmaf(wb.y, re, acc[r].y);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
    }

    if (pvalid) {
        float2* out = G + (static_cast<size_t>(py) * a.nx + px) * a.n_z;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int kz = blk * KB + wave * RW + r;
            if (kz < a.n_z) out[kz] = acc[r];
        }
    }
}

template <int KB, int RSC>
__global__ __launch_bounds__(64 * kGatherWaves) void backproject_gather_kernel(const float2* __restrict__ q,
                                                                               const GatherTileEntry* __restrict__ tab,
                                                                               BpgArgs a, float2* __restrict__ G) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int work = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    if (work >= a.n_work) return;  // workgroup-uniform, before any barrier
    const int blk = work / a.n_tiles;
    gather_tile<KB, RSC>(a, q, tab, G, blk, work - blk * a.n_tiles, smem);
}

struct TileTableArgs {
    int n_ch, n_l, tiles_x, n_tiles, tile_x, tile_y, wpl, n_blocks;
    double x0, y0, dx, dy, inv_du, reach;
    double kref[kMaxBlocks];
};

// The tile table (see GatherTileEntry), one thread per (tile, channel): the
// tile's centre, its range from the channel's antennas in float64, the
// even start of the channel's staged window (wpl samples) and the centre's
// first tap and fractional position relative to it; then the centre's
// carrier for every k_z block (after the entries).
__global__ void tile_table_kernel(TileTableArgs a, const double* __restrict__ chan, const double* __restrict__ llo,
                                  GatherTileEntry* __restrict__ tab) {
    float2* carr = reinterpret_cast<float2*>(tab + static_cast<size_t>(a.n_tiles) * a.n_ch);
    const long long n = static_cast<long long>(a.n_tiles) * a.n_ch;
    for (long long e = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; e < n;
         e += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int tile = static_cast<int>(e / a.n_ch), c = static_cast<int>(e - static_cast<long long>(tile) * a.n_ch);
        const int tx0 = (tile % a.tiles_x) * a.tile_x, ty0 = (tile / a.tiles_x) * a.tile_y;
        const double cx = a.x0 + (tx0 + 0.5 * (a.tile_x - 1)) * a.dx, cy = a.y0 + (ty0 + 0.5 * (a.tile_y - 1)) * a.dy;
        const double* ch = chan + 4 * c;
        const double xt = cx - ch[0], yt = cy - ch[1], xr = cx - ch[2], yr = cy - ch[3];
        const double dt = sqrt(xt * xt + yt * yt), dr = sqrt(xr * xr + yr * yr);
        const double l = dt + dr;
        int s = static_cast<int>(floor((l - a.reach - llo[c]) * a.inv_du)) - 2;
        s = max(0, min(s, a.n_l - a.wpl)) & ~1;
        const double u = (l - llo[c]) * a.inv_du;
        const double fl = floor(u);
        GatherTileEntry t;
        t.lc = l;
        t.win = s;
        t.base = static_cast<int>(fl) - 1 - s;
        t.uf = static_cast<float>(u - fl);
        t.xt = static_cast<float>(xt);
        t.yt = static_cast<float>(yt);
        t.dt = static_cast<float>(dt);
        t.xr = static_cast<float>(xr);
        t.yr = static_cast<float>(yr);
        t.dr = static_cast<float>(dr);
        t.pad_ = 0.f;
        tab[e] = t;
        for (int b = 0; b < a.n_blocks; ++b)
            carr[(static_cast<size_t>(b) * a.n_tiles + tile) * a.n_ch + c] = cis_rev(a.kref[b] * (0.5 / kPi) * l);
    }
}

// Persistent form for a batch of scans: eight work queues, one per XCD, each
// a contiguous range [bounds[x], bounds[x+1]) of (scan, k_z block, tile)
// items (cost-balanced, heaviest scans first) with an atomic counter.  A
// workgroup takes items from its own XCD's queue (so an XCD's L2 sees a
// compact set of range profiles) and, once it is empty, from the others in
// turn; it leaves after all eight are exhausted.
// wsr and ws are the same batch workspace: wsr for what the kernel only
// reads (range profiles, tile tables), ws for the spectra it writes; the
// regions are disjoint, and the separate restrict views let the tile-table
// reads use scalar loads.
template <int KB, int RSC>
__global__ __launch_bounds__(64 * kGatherWaves) void backproject_gather_batch_kernel(
    const BatchScanDesc* __restrict__ scans, const int4* __restrict__ items, const int* __restrict__ bounds,
    unsigned* __restrict__ counters, const char* __restrict__ wsr, char* __restrict__ ws) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    // the item index travels in the first word of the weight slots, which
    // are free between items (no static LDS: it would cost a workgroup per
    // CU at row lengths that fill the LDS exactly)
    int* next = reinterpret_cast<int*>(smem);
    const int home = blockIdx.x & 7;
    for (int k = 0; k < 8; ++k) {
        const int x = (home + k) & 7;
        const int lo = bounds[x], hi = bounds[x + 1];
        for (;;) {
            if (threadIdx.x == 0) *next = lo + static_cast<int>(atomicAdd(counters + x, 1u));
            __syncthreads();
            // wavefront-uniform (readfirstlane): the item's scan, block and
            // tile then address the descriptors and tile tables with scalar loads
            const int it = __builtin_amdgcn_readfirstlane(*next);
            __syncthreads();  // every thread has read `next` before it is overwritten
            if (it >= hi) break;
            const int4 w = items[it];
            const int sc = __builtin_amdgcn_readfirstlane(w.x), blk = __builtin_amdgcn_readfirstlane(w.y),
                      tile = __builtin_amdgcn_readfirstlane(w.z);
            const BatchScanDesc& d = scans[sc];
            gather_tile<KB, RSC>(d.a, reinterpret_cast<const float2*>(wsr + d.q_off),
                                 reinterpret_cast<const GatherTileEntry*>(wsr + d.tab_off),
                                 reinterpret_cast<float2*>(ws + d.g_off), blk, tile, smem);
            __syncthreads();  // LDS is reused by the next item
        }
    }
}

__global__ void reset_counters_kernel(unsigned* c) {
    if (threadIdx.x < 8) c[threadIdx.x] = 0u;
}

template <int KB, int RSC>
int launch_gather(const BpgArgs& a, size_t smem, unsigned blocks, hipStream_t s, const float2* q,
                  const GatherTileEntry* tab, float2* G) {
    auto fn = backproject_gather_kernel<KB, RSC>;
    if (smem > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem));
        if (e != hipSuccess) return fail(PL_EDEVICE, "back-projection LDS of %zu bytes: %s", smem, hipGetErrorString(e));
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * kGatherWaves), smem, s, q, tab, a, G);
    return check_launch("back-projection (pixel per lane)");
}

BpgArgs gather_args(const HybridPlan& p) {
    BpgArgs a{};
    a.n_ch = p.n_ch;
    a.n_z = p.n_z;
    a.n_l = p.n_l;
    a.nx = p.nx;
    a.ny = p.ny;
    a.tiles_x = p.tiles_x;
    a.n_tiles = p.tiles_x * p.tiles_y;
    a.n_work = a.n_tiles * p.n_blocks;
    a.per_xcd = (a.n_work + 7) / 8;
    a.nchk = p.window / 2;  // staged chunks: the window
    a.mono = p.mode == PL_MONO;
    a.x0 = p.x0;
    a.y0 = p.y0;
    a.dx = p.dx;
    a.dy = p.dy;
    a.inv_du = 1.0 / p.du;
    a.reach = std::hypot(7.0 * p.dx, 7.0 * p.dy);  // 2 x half-diagonal of the 8x8 tile
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 4; ++j) a.coef[k][j] = p.coef[k][j];
    for (int b = 0; b < kMaxBlocks; ++b) a.kref[b] = p.kref[b];
    return a;
}

int check_gather_plan(const HybridPlan& p, int rsc) {
    const int nchk = p.window / 2;
    if (!p.bp_gather || (p.block != 32 && p.block != 64) || p.tile_x != 8 || p.tile_y != 8 || p.window % 2 ||
        nchk < 3 || nchk > p.window_pad || p.window_pad > rsc || 2 * nchk > p.n_l || p.waves != kGatherWaves)
        return fail(PL_EUNSUPPORTED, "pixel-per-lane back-projection: window %d, block %d", p.window, p.block);
    // one channel's profiles are addressed by a 32-bit buffer descriptor
    if (static_cast<unsigned long long>(p.n_z) * p.n_l * 8 >= (1ull << 31))
        return fail(PL_EUNSUPPORTED, "range profiles of one channel exceed 2 GiB");
    return PL_OK;
}

// Compiled (k_z bins, row chunks) classes of the pixel-per-lane kernels; the
// row lengths are the longest at each occupancy level with 32 bins (LDS
// 8 KiB + 2 KiB per chunk: 8, 7, 6, 5, 4 and 3 workgroups per CU).
#define PL_GATHER_CLASSES(X) \
    X(64, 12) X(64, 14) X(64, 18) X(64, 24) X(64, 32) X(64, 40) X(32, 12) X(32, 14) X(32, 18) X(32, 24) X(32, 32) X(32, 40)

template <int KB, int RSC>
const void* gather_batch_fn() {
    return reinterpret_cast<const void*>(backproject_gather_batch_kernel<KB, RSC>);
}

const void* gather_batch_kernel(int kb, int rsc) {
#define PL_GB(KB, RSC) \
    if (kb == KB && rsc == RSC) return gather_batch_fn<KB, RSC>();
    PL_GATHER_CLASSES(PL_GB)
#undef PL_GB
    return nullptr;
}

int run_gather(const HybridPlan& p, const DeviceTables& dt, const float2* q, char* ws, float2* G, hipStream_t s) {
    const BpgArgs a = gather_args(p);
    int rc = check_gather_plan(p, p.window_pad);
    if (rc) return rc;
    const size_t smem = backproject_gather_lds_bytes(p.block, p.window_pad);
    if (smem > kMaxLds) return fail(PL_EUNSUPPORTED, "back-projection needs %zu bytes of LDS", smem);
    const unsigned blocks = static_cast<unsigned>(8 * a.per_xcd);
    const GatherTileEntry* tab = reinterpret_cast<const GatherTileEntry*>(ws + p.off_tiles);
    (void)dt;
#define PL_G(KB, RSC) \
    if (p.block == KB && p.window_pad == RSC) return launch_gather<KB, RSC>(a, smem, blocks, s, q, tab, G);
    PL_GATHER_CLASSES(PL_G)
#undef PL_G
    return fail(PL_EUNSUPPORTED, "no pixel-per-lane back-projection for %d-chunk rows", p.window_pad);
}

}  // namespace

size_t gather_batch_desc_bytes() { return sizeof(BatchScanDesc); }

int build_gather_batch_desc(const HybridPlan& p, size_t ws_off, int rsc, void* out) {
    int rc = check_gather_plan(p, rsc);
    if (rc) return rc;
    BatchScanDesc d{};
    d.a = gather_args(p);
    d.q_off = ws_off + p.off_q;
    d.tab_off = ws_off + p.off_tiles;
    d.g_off = ws_off + p.off_G;
    std::memcpy(out, &d, sizeof(d));
    return PL_OK;
}

int gather_batch_grid(int kb, int rsc, size_t smem, int* blocks) {
    const void* fn = gather_batch_kernel(kb, rsc);
    if (!fn) return fail(PL_EUNSUPPORTED, "no batched back-projection for %d k_z bins, %d-chunk rows", kb, rsc);
    if (smem > kMaxLds) return fail(PL_EUNSUPPORTED, "batched back-projection needs %zu bytes of LDS", smem);
    if (smem > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem)) !=
                            hipSuccess)
        return fail(PL_EDEVICE, "batched back-projection: LDS of %zu bytes refused", smem);
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kGatherWaves, smem) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(PL_EDEVICE, "batched back-projection: occupancy query failed");
    // Workgroups beyond the resident ones start only once the queues are
    // empty and leave at once, so size the grid by the LDS bound too.
    const int by_lds = static_cast<int>(kMaxLds / (smem + 256));
    *blocks = (std::max(1, std::max(per_cu, std::min(by_lds, 8))) * cus + 7) & ~7;
    return PL_OK;
}

int launch_gather_batch(const void* descs, const void* items, const int* bounds, unsigned* counters, char* ws,
                        int kb, int rsc, size_t smem, int blocks, hipStream_t s) {
    const void* fn = gather_batch_kernel(kb, rsc);
    if (!fn) return fail(PL_EUNSUPPORTED, "no batched back-projection for %d k_z bins, %d-chunk rows", kb, rsc);
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, counters);
    int rc = check_launch("batch work counters");
    if (rc) return rc;
    auto args_descs = static_cast<const BatchScanDesc*>(descs);
    auto args_items = static_cast<const int4*>(items);
#define PL_GB(KB, RSC)                                                                                          \
    if (kb == KB && rsc == RSC) {                                                                               \
        hipLaunchKernelGGL((backproject_gather_batch_kernel<KB, RSC>), dim3(blocks), dim3(64 * kGatherWaves), smem, \
                           s, args_descs, args_items, bounds, counters, ws, ws);                                \
        return check_launch("batched back-projection");                                                         \
    }
    PL_GATHER_CLASSES(PL_GB)
#undef PL_GB
    return fail(PL_EUNSUPPORTED, "no batched back-projection for %d k_z bins, %d-chunk rows", kb, rsc);
}

size_t backproject_gather_lds_bytes(int rows, int row_chunks) {
    return 1ull * kGatherBatch * 2 * 64 * 16 + 2ull * rows * row_chunks * 16;
}

size_t tile_table_bytes(const HybridPlan& p) {
    return (p.bp_gather || p.bp_mfma)
               ? static_cast<size_t>(p.tiles_x) * p.tiles_y * p.n_ch * (sizeof(GatherTileEntry) + p.n_blocks * sizeof(float2))
               : 0;
}

int launch_tile_tables(const HybridPlan& p, const DeviceTables& dt, char* ws, hipStream_t s) {
    if (!p.bp_gather && !p.bp_mfma) return PL_OK;
    TileTableArgs a{};
    a.n_ch = p.n_ch;
    a.n_l = p.n_l;
    a.tiles_x = p.tiles_x;
    a.n_tiles = p.tiles_x * p.tiles_y;
    a.tile_x = p.tile_x;
    a.tile_y = p.tile_y;
    a.wpl = p.bp_gather ? p.window : 8 * (p.window / 8);  // staged samples per row (plane)
    a.x0 = p.x0;
    a.y0 = p.y0;
    a.dx = p.dx;
    a.dy = p.dy;
    a.inv_du = 1.0 / p.du;
    a.reach = std::hypot((p.tile_x - 1) * p.dx, (p.tile_y - 1) * p.dy);  // 2 x the tile's half-diagonal
    a.n_blocks = p.n_blocks;
    for (int b = 0; b < kMaxBlocks; ++b) a.kref[b] = p.kref[b];
    const long long n = static_cast<long long>(a.n_tiles) * a.n_ch;
    const int blocks = static_cast<int>(std::min<long long>((n + 255) / 256, 8192));
    hipLaunchKernelGGL(tile_table_kernel, dim3(blocks), dim3(256), 0, s, a, dt.chan,
                       reinterpret_cast<const double*>(ws + p.off_llo), reinterpret_cast<GatherTileEntry*>(ws + p.off_tiles));
    return check_launch("back-projection tile table");
}

size_t backproject_lds_bytes(int n_ch, int rows, int window_pad) {
    return static_cast<size_t>((n_ch + 63) & ~63) * 4 + 2ull * rows * window_pad * 8;
}

int launch_backproject(const HybridPlan& p, const DeviceTables& dt, const float2* q, char* ws, float2* G,
                       hipStream_t s) {
    if (p.bp_gather) return run_gather(p, dt, q, ws, G, s);
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
    a.rows = p.block;
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
    if (static_cast<unsigned long long>(p.n_z) * p.n_l * 8 >= (1ull << 31))
        return fail(PL_EUNSUPPORTED, "range profiles of one channel exceed 2 GiB");
    if (p.window < 4 || p.window > 128 || p.window > p.n_l)
        return fail(PL_EUNSUPPORTED, "back-projection window %d out of range", p.window);
    const size_t smem = backproject_lds_bytes(p.n_ch, p.block, p.window_pad);
    if (smem > kMaxLds) return fail(PL_EUNSUPPORTED, "back-projection needs %zu bytes of LDS", smem);
    const unsigned blocks = static_cast<unsigned>(8 * a.per_xcd);
    const double* llo = reinterpret_cast<const double*>(ws + p.off_llo);
    const double* krz = reinterpret_cast<const double*>(ws + p.off_krz);
    const int kpl = p.block / kLanes;
    if (p.ref_mode == PL_REF_MIN_K) {
        if (kpl != 1 || p.waves != 4)
            return fail(PL_EUNSUPPORTED, "per-k_z references run one k_z bin per lane, 4 wavefronts");
        if (p.tile_x == 8 && p.tile_y == 8) return launch_variant<8, 8, 1, 4, 4, true>(a, smem, blocks, s, q, dt.chan, llo, krz, G);
        if (p.tile_x == 4 && p.tile_y == 4) return launch_variant<4, 4, 1, 4, 4, true>(a, smem, blocks, s, q, dt.chan, llo, krz, G);
        if (p.tile_x == 2 && p.tile_y == 2) return launch_variant<2, 2, 1, 4, 4, true>(a, smem, blocks, s, q, dt.chan, llo, krz, G);
        return fail(PL_EUNSUPPORTED, "no per-k_z-reference back-projection for tile %dx%d", p.tile_x, p.tile_y);
    }
#define PL_CASE(TX, TY, K, NW, OCC)                                                   \
    if (p.tile_x == TX && p.tile_y == TY && kpl == K && p.waves == NW)                \
        return launch_variant<TX, TY, K, NW, OCC>(a, smem, blocks, s, q, dt.chan, llo, krz, G);
    PL_CASE(8, 8, 1, 4, 4) PL_CASE(8, 8, 2, 4, 2) PL_CASE(8, 8, 4, 4, 1)
    PL_CASE(8, 8, 1, 8, 4) PL_CASE(8, 8, 2, 8, 4) PL_CASE(8, 8, 4, 8, 2)
    PL_CASE(4, 4, 1, 4, 4) PL_CASE(4, 4, 2, 4, 2) PL_CASE(4, 4, 4, 4, 1)
    PL_CASE(2, 2, 1, 4, 4) PL_CASE(2, 2, 2, 4, 2) PL_CASE(2, 2, 4, 4, 1)
#undef PL_CASE
    return fail(PL_EUNSUPPORTED, "no back-projection kernel for tile %dx%d, %d k_z per lane, %d waves", p.tile_x,
                p.tile_y, kpl, p.waves);
}

}  // namespace pl
