// Back-projection onto horizontal-plane pixels, eq. (8b) / (19b), on the
// matrix cores (BF16 / FP16 modes).
//
// For one channel c, a 4x4 pixel group and 16 k_z bins the interpolation is a
// small dense product over a 16-sample window of the range grid:
//   G[kz][p] += sum_s Q_c[kz][s] B_c[s][p],
//   B_c[s][p] = K(x_p - s) exp(j k_ref l_c(p)),
// with x_p the pixel's position in the window and K the 4-tap interpolation
// kernel.  With the real embedding A = [Re Q | Im Q] (16 kz x 32):
//   Re G = A [Re B; -Im B],   Im G = A [Im B; Re B],
// one v_mfma_f32_16x16x32_bf16 each per split product; operands are BF16
// hi + lo parts and each pair takes hi*hi + hi*lo + lo*hi (FP32 accumulation).
//
// Workgroup = TX x TY pixel tile (4x4 groups, GPW per wavefront, NW wavefronts) x KB k_z
// bins sharing one reference wavenumber.  The range profiles arrive split
// (four BF16 planes per (channel, k_z): Re hi, Re lo, Im hi, Im lo).  For
// each channel the tile's window rows are copied into LDS by 16-byte direct
// global-to-LDS loads, one channel ahead (double buffer, one barrier per
// channel).
//
// LDS row of one k_z bin: 33 chunks of 16 bytes; plane p occupies chunks
// [8p, 8p + 8) (its first nck chunks hold the window, nck <= 8) and chunk 32
// is padding.  A half-wave's A-operand read (16 rows x 2 lane groups x 8
// bytes) then falls on distinct banks whether the LDS serves 32 or 64 lanes
// per cycle: the row stride is an odd number of chunks and the imaginary
// planes sit 256 bytes after the real ones.  All read offsets are constants.
//
// K-index order: lane group kg = lane / 16 of an operand holds samples
// {4h .. 4h+3, 8+4h .. 8+4h+3} (h = kg & 1) of the real (kg < 2) or the
// imaginary (kg >= 2) plane, so each A fragment is two aligned 8-byte reads.
//
// Single-pass form (SP): the profiles arrive as two FP16 planes per
// (channel, k_z), Re and Im, scaled by one power of two 2^-g for the whole
// call so that every value lies below 2^15 (the scale and g are set by the
// range compression).  The operand B is rounded once to FP16 and each pair
// takes one v_mfma_f32_16x16x32_f16 per output part (FP32 accumulation); the
// result is multiplied by 2^g.  LDS rows are 17 chunks: Re in [0, 8), Im in
// [8, 16), chunk 16 padding.  Each product then carries two FP16 roundings
// (relative 2^-11 each) instead of the split form's FP32-class error.
#include <algorithm>
#include <atomic>
#include <cstring>

#include "device.hpp"

namespace pl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kRowChunks = 33;              // 16-byte chunks per LDS row (split form)
constexpr int kRowChunksSP = 17;            // single-pass form
constexpr int kPlaneBytes = 128;            // 8 chunks per plane
__host__ __device__ constexpr int row_chunks(bool sp) { return sp ? kRowChunksSP : kRowChunks; }
// channels staged per barrier: two in the single-pass form with 64 k_z bins
// (its rows are half as long, so two channels' double buffers still fit two
// workgroups per CU), else one
__host__ __device__ constexpr int stage_channels(bool sp, int kz_block) { return sp && kz_block == 64 ? 2 : 1; }
constexpr int kSelEntries = 20;             // selector table: a0 = 4h - d0 in [-15, 4]

struct BpmArgs {
    int n_ch, n_z, n_l, nx, ny, tiles_x, n_tiles, n_work, per_xcd, nck, mono;
    // Work items [0, n_whole) run whole, on the first grid_whole workgroups
    // (per_xcd per XCD); each later item is split into n_part pieces of
    // whole groups of four channels (n_ch4 groups), one workgroup each
    // (per_xcd_tail per XCD, in (item, piece) order), that write partial
    // spectra to part (see the tail split at launch_cfg).
    int n_whole, grid_whole, n_part, n_ch4, per_xcd_tail;
    float2* part;
    const int* qexp;  // single-pass form: the profiles' scale exponent g
    double x0, y0, dx, dy, inv_du;
    float coef[4][4];  // tap j weight = sum_k coef[j][k] t^k, taps at floor(u) - 1 + j
    double kref[kMaxBlocks];
};

// Two floats to a packed BF16 pair (round to nearest even), one instruction.
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2{lo, hi}), bf16x2));
}

// Two floats to a packed FP16 pair (round to nearest even), one instruction.
__device__ __forceinline__ unsigned pack_f16(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2{lo, hi}), f16x2));
}

// Split x = hi + lo for the two values packed in h (BF16 pair of (x0, x1)).
__device__ __forceinline__ unsigned pack_lo(float x0, float x1, unsigned h) {
    return pack_bf16(x0 - __uint_as_float(h << 16), x1 - __uint_as_float(h & 0xffff0000u));
}

// v_perm selector bytes of tap k (two bytes of a BF16 value) or zero bytes.
__host__ __device__ constexpr unsigned tap_sel(int k) {
    return (k >= 0 && k < 4) ? 0x0100u + 0x0202u * static_cast<unsigned>(k) : 0x0c0cu;
}

// 16-byte direct global-to-LDS copy.  The 16-byte form of the builtin exists
// for the device target only; the host pass of this translation unit, which
// emits the launch stubs, must not see it.
#if defined(__HIP_DEVICE_COMPILE__)
#define PL_DMA16(SRC, DST) __builtin_amdgcn_global_load_lds((SRC), (DST), 16, 0, 0)
#else
#define PL_DMA16(SRC, DST) ((void)(SRC), (void)(DST))
#endif

// Window start of a tile-table entry through the constant address space: a
// scalar load (lgkmcnt), so that taking it never waits for the row copies in
// flight (vmcnt), as a vector load would.  The address is wavefront-uniform.
__device__ __forceinline__ int entry_win(const GatherTileEntry* e) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *reinterpret_cast<const __attribute__((address_space(4))) int*>(reinterpret_cast<unsigned long long>(&e->win));
#else
    return e->win;
#endif
}

// This wavefront's share of one channel's window rows: instruction
// i = wave + NW j fills LDS chunks [64 i, 64 i + 64) of the buffer at DST0;
// lanes whose chunk is padding or beyond the window (doff = ~0) are idle.
#define PL_STAGE_ROWS(BASE, DST0)                                                  \
    do {                                                                           \
        const char* base_ = (BASE);                                                \
        unsigned char* dst0_ = (DST0);                                             \
        _Pragma("unroll") for (int j_ = 0; j_ < NIW; ++j_) {                        \
            const int i_ = wave + NW * j_;                                         \
            if (i_ * 64 < KB * RC && doff[j_] != ~0u)                              \
                PL_DMA16(base_ + doff[j_], dst0_ + i_ * 1024);                     \
        }                                                                          \
    } while (0)

// Eight-wavefront workgroups aim at four wavefronts per SIMD (two
// workgroups per CU), which caps a wavefront at 128 registers.
template <int GPW, int KT, int NW, bool SP>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 8 ? 4 : 1)))
void backproject_mfma_kernel(const unsigned short* __restrict__ qs, const GatherTileEntry* __restrict__ tab,
                             BpmArgs a, float2* __restrict__ G) {
    constexpr int KB = 16 * KT;
    constexpr int NG = GPW * NW;                                    // groups per tile
    constexpr int GX = NG == 4 ? 2 : 4, GY = NG / GX;
    static_assert(NG == 4 || NG == 8 || NG == 16, "8x8, 16x8 or 16x16 pixel tiles");
    constexpr int TX = 4 * GX, TY = 4 * GY;
    constexpr int RC = row_chunks(SP), RB = 16 * RC, NP = SP ? 2 : 4;  // row chunks, row bytes, planes
    constexpr int NIW = (KB * RC + 64 * NW - 1) / (64 * NW);  // DMA instructions per wavefront
    constexpr unsigned kBufBytes = KB * RB;
    constexpr int CPS = stage_channels(SP, KB);
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    u32x4* sel_tab = reinterpret_cast<u32x4*>(smem);
    constexpr unsigned lds0 = kSelEntries * 16;

    // this workgroup's work item and channels [cb, ce) (workgroup-uniform;
    // the returns come before any barrier)
    int work, piece = -1, cb = 0, ce = a.n_ch;
    if (static_cast<int>(blockIdx.x) < a.grid_whole) {
        work = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
        if (work >= a.n_whole) return;
    } else {
        const int bt = blockIdx.x - a.grid_whole;
        piece = (bt & 7) * a.per_xcd_tail + (bt >> 3);   // a contiguous share per XCD
        if (piece >= (a.n_work - a.n_whole) * a.n_part) return;
        const int part = piece % a.n_part;
        work = a.n_whole + piece / a.n_part;
        cb = 4 * (part * a.n_ch4 / a.n_part);   // a multiple of four: the batches and
        ce = min(a.n_ch, 4 * ((part + 1) * a.n_ch4 / a.n_part));   // stage buffers line up
    }
    const int blk = work / a.n_tiles;
    const int tile = work - blk * a.n_tiles;
    const int tx0 = (tile % a.tiles_x) * TX, ty0 = (tile / a.tiles_x) * TY;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wpl = 8 * a.nck;  // staged samples per plane
    const float kref_rev_f = static_cast<float>(a.kref[blk] * (0.5 / kPi));
    const float inv_du_f = static_cast<float>(a.inv_du);
    const GatherTileEntry* tt = tab + static_cast<size_t>(tile) * a.n_ch;
    // the tile centres' carriers of this k_z block (after the table's entries)
    const float2* tc = reinterpret_cast<const float2*>(tab + static_cast<size_t>(a.n_tiles) * a.n_ch) +
                       (static_cast<size_t>(blk) * a.n_tiles + tile) * a.n_ch;

    // selectors of the sample pairs (a, a+1), (a+2, a+3), (a+8, a+9),
    // (a+10, a+11) in tap units, a = a0 = 4h - d0, entry a0 + 15
    if (tid < kSelEntries) {
        const int a0 = tid - 15;
        u32x4 e;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int k = a0 + 2 * (o & 1) + 8 * (o >> 1);
            e[o] = tap_sel(k) | (tap_sel(k + 1) << 16);
        }
        sel_tab[tid] = e;
    }

    // Per-lane byte offsets of this wavefront's DMA chunks (relative to the
    // channel's window start), ~0 for idle lanes.
    unsigned doff[NIW];
#pragma unroll
    for (int j = 0; j < NIW; ++j) {
        const int g = (wave + NW * j) * 64 + lane;
        const int r = g / RC, jj = g - r * RC;
        const int part = jj >> 3, k8 = jj & 7;
        const int kz = min(blk * KB + r, a.n_z - 1);
        doff[j] = (r < KB && jj < 8 * NP && k8 < a.nck)
                      ? static_cast<unsigned>(((kz * NP + part) * a.n_l + 8 * k8) * 2)
                      : ~0u;
    }
    const size_t chan_elems = static_cast<size_t>(a.n_z) * NP * a.n_l;

    // pixel pn of each group (the operand column of this lane), its offset
    // from the tile centre; k' group of the MFMA operands
    const int pn = lane & 15, kg = lane >> 4, h = kg & 1;
    int gpx[GPW], gpy[GPW];
    float ox[GPW], oy[GPW];
#pragma unroll
    for (int g = 0; g < GPW; ++g) {
        const int gi = wave * GPW + g;
        const int lx = 4 * (gi % GX) + (pn & 3), ly = 4 * (gi / GX) + (pn >> 2);
        gpx[g] = tx0 + lx;
        gpy[g] = ty0 + ly;
        ox[g] = (lx - 0.5f * (TX - 1)) * static_cast<float>(a.dx);
        oy[g] = (ly - 0.5f * (TY - 1)) * static_cast<float>(a.dy);
    }

    f32x4 accr[GPW][KT], acci[GPW][KT];
#pragma unroll
    for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int t = 0; t < KT; ++t) {
            accr[g][t] = f32x4{0.f, 0.f, 0.f, 0.f};
            acci[g][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        }

    // channel c's rows go to buffer (c / CPS) % 2 * CPS + c % CPS (cb is a
    // multiple of 2 CPS, so the first channel takes buffer 0)
#pragma unroll
    for (int k = 0; k < CPS; ++k)
        if (cb + k < ce)
            PL_STAGE_ROWS(reinterpret_cast<const char*>(qs + (cb + k) * chan_elems + entry_win(tt + cb + k)),
                          smem + lds0 + k * kBufBytes);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // selector table and the first channels' rows visible

    // LDS byte offset of this lane's A operand within a buffer: row m = lane
    // & 15 of a k_z tile, hi plane (split: 0 real, 2 imaginary; SP: 0, 1),
    // samples 4h.. of the group window; the lo plane is kPlaneBytes further
    const unsigned a_lane = static_cast<unsigned>(pn * RB) + (kg < 2 ? 0u : (SP ? 1u : 2u) * kPlaneBytes) + 8u * h;
    // Each 8-byte piece of an A fragment is read from its own base register
    // (offsets the compiler cannot see): adjacent pieces would otherwise be
    // merged into ds_read2_b64, which serves fewer lanes per cycle, and rows
    // 4 dwords apart then share banks.  A separate ds_read_b64 serves half a
    // wavefront per cycle, conflict-free in this layout.
    unsigned dq[3] = {16u, kPlaneBytes, kPlaneBytes + 16u};
    asm volatile("" : "+v"(dq[0]), "+v"(dq[1]), "+v"(dq[2]));

#pragma unroll 1
    for (int c0 = cb; c0 < ce; c0 += 4) {
        // Geometry of the batch: lane (k = lane / 16, pn) takes pixel pn of
        // each group and channel c0 + k: its range from the tile table
        // (float64 centre, float32 offset), its position in the group's
        // 16-sample window and its carrier; the MFMA lanes (pn, kg) of
        // channel c0 + cc read them from lane 16 cc + pn.  The single-pass
        // form also forms the pixel's four tap weights times the carrier
        // here, packed to FP16 (P = w Re c, Q = w Im c), once per (pixel,
        // channel) instead of once per MFMA lane.
        float xw[GPW], crw[GPW], ciw[GPW];
        unsigned pw0[GPW], pw1[GPW], qw0[GPW], qw1[GPW];
        int dw[GPW], srw[GPW];
        {
            const int c = min(c0 + (lane >> 4), a.n_ch - 1);
            const GatherTileEntry e = tt[c];
            const float2 cc0 = tc[c];   // the centre's carrier (float64 phase, in the table)
#pragma unroll
            for (int g = 0; g < GPW; ++g) {
                const bool ok = gpx[g] < a.nx && gpy[g] < a.ny;
                const float oo = ox[g] * ox[g] + oy[g] * oy[g];
                const float sT = 2.f * (e.xt * ox[g] + e.yt * oy[g]) + oo;
                float dl = sT * __builtin_amdgcn_rcpf(e.dt + __builtin_amdgcn_sqrtf(e.dt * e.dt + sT));
                if (a.mono) {
                    dl += dl;
                } else {
                    const float sR = 2.f * (e.xr * ox[g] + e.yr * oy[g]) + oo;
                    dl += sR * __builtin_amdgcn_rcpf(e.dr + __builtin_amdgcn_sqrtf(e.dr * e.dr + sR));
                }
                const float uu = e.uf + dl * inv_du_f;
                const float fv = floorf(uu);
                const int i0 = e.base + static_cast<int>(fv);   // first tap, from the window start
                int m = ok ? i0 : 0x3fffffff;
                m = min(m, __shfl_xor(m, 1));
                m = min(m, __shfl_xor(m, 2));
                m = min(m, __shfl_xor(m, 4));
                m = min(m, __shfl_xor(m, 8));
                const int sr = m == 0x3fffffff ? 0 : max(0, min(m & ~3, wpl - 16));
                srw[g] = sr;
                const float2 c1 = cis_rev_f(kref_rev_f * dl);   // |dl| spans a tile: a few revolutions
                const float cr = ok ? cc0.x * c1.x - cc0.y * c1.y : 0.f;
                const float ci = ok ? cc0.x * c1.y + cc0.y * c1.x : 0.f;
                if constexpr (SP) {
                    const float t = uu - fv;
                    float w[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        w[j] = ((a.coef[j][3] * t + a.coef[j][2]) * t + a.coef[j][1]) * t + a.coef[j][0];
                    pw0[g] = pack_f16(w[0] * cr, w[1] * cr);
                    pw1[g] = pack_f16(w[2] * cr, w[3] * cr);
                    qw0[g] = pack_f16(w[0] * ci, w[1] * ci);
                    qw1[g] = pack_f16(w[2] * ci, w[3] * ci);
                    dw[g] = ok ? i0 - sr : 1000;   // first tap in the group window
                } else {
                    // position in the group window: floor(x) - 1 is the first tap
                    xw[g] = ok ? static_cast<float>(i0 - sr + 1) + (uu - fv) : 1000.f;
                    crw[g] = cr;
                    ciw[g] = ci;
                }
            }
        }
#pragma unroll 1
        for (int cc = 0; cc < 4; ++cc) {
            const int c = c0 + cc;
            if (c >= ce) break;
            if (c % CPS == 0) {   // the next stage's channels, into the other buffers
#pragma unroll
                for (int k = 0; k < CPS; ++k) {
                    const int cn = c + CPS + k;
                    if (cn < ce)
                        PL_STAGE_ROWS(reinterpret_cast<const char*>(qs + cn * chan_elems + entry_win(tt + cn)),
                                      smem + lds0 + (((cn / CPS) & 1) * CPS + k) * kBufBytes);
                }
            }
            const unsigned bufo = lds0 + (((c / CPS) & 1) * CPS + c % CPS) * kBufBytes;
            const int src = cc * 16 + pn;
#pragma unroll
            for (int g = 0; g < GPW; ++g) {
                const int sr = __builtin_amdgcn_readlane(srw[g], cc * 16);
                const unsigned char* ap = smem + bufo + a_lane + 2u * static_cast<unsigned>(sr);
                if constexpr (SP) {
                    // B operand: the pixel's packed taps times the carrier,
                    // placed at this lane's 8 samples by byte permutes.  Rows
                    // of Re Q (kg < 2) take P = Re B for Re G and Q = Im B
                    // for Im G; rows of Im Q take -Q for Re G and P for Im G
                    // (the sign flip of packed FP16 is exact)
                    const unsigned p0 = __shfl(pw0[g], src), p1 = __shfl(pw1[g], src);
                    const unsigned q0 = __shfl(qw0[g], src), q1 = __shfl(qw1[g], src);
                    const int d0 = __shfl(dw[g], src);
                    const int a0 = min(max(4 * h - d0, -15), 4);   // a0 = 4h - d0, d0 the first tap
                    const u32x4 sel = sel_tab[a0 + 15];
                    const unsigned rh0 = kg < 2 ? p0 : q0 ^ 0x80008000u, rh1 = kg < 2 ? p1 : q1 ^ 0x80008000u;
                    const unsigned ih0 = kg < 2 ? q0 : p0, ih1 = kg < 2 ? q1 : p1;
                    u32x4 vr, vi;
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        vr[o] = __builtin_amdgcn_perm(rh1, rh0, sel[o]);
                        vi[o] = __builtin_amdgcn_perm(ih1, ih0, sel[o]);
                    }
                    const f16x8 br = __builtin_bit_cast(f16x8, vr), bi = __builtin_bit_cast(f16x8, vi);
                    // every k_z tile's A fragment first, then the products:
                    // one wait for the LDS reads instead of one per tile
                    f16x8 va[KT];
#pragma unroll
                    for (int t = 0; t < KT; ++t) {
                        const u32x2 h0 = *reinterpret_cast<const u32x2*>(ap + t * 16 * RB);
                        const u32x2 h1 = *reinterpret_cast<const u32x2*>(ap + dq[0] + t * 16 * RB);
                        va[t] = __builtin_bit_cast(f16x8, u32x4{h0[0], h0[1], h1[0], h1[1]});
                    }
#pragma unroll
                    for (int t = 0; t < KT; ++t) {
                        accr[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(va[t], br, accr[g][t], 0, 0, 0);
                        acci[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(va[t], bi, acci[g][t], 0, 0, 0);
                    }
                } else {
                    // B operand: taps of this lane's pixel times the carrier,
                    // placed at its 8 samples by byte permutes
                    const float xn = __shfl(xw[g], src), crn = __shfl(crw[g], src), cin = __shfl(ciw[g], src);
                    const float fl = floorf(xn);
                    const float t = xn - fl;
                    // a0 = 4h - d0 with d0 = floor(x) - 1 the first tap in the group window
                    const int a0 = min(max(4 * h + 1 - static_cast<int>(fl), -15), 4);
                    const u32x4 sel = sel_tab[a0 + 15];
                    float w[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        w[j] = ((a.coef[j][3] * t + a.coef[j][2]) * t + a.coef[j][1]) * t + a.coef[j][0];
                    const float ca = kg < 2 ? crn : -cin;  // rows of Re Q: Re B (Re G), Im B (Im G)
                    const float cb = kg < 2 ? cin : crn;   // rows of Im Q: -Im B, Re B
                    const float r0 = w[0] * ca, r1 = w[1] * ca, r2 = w[2] * ca, r3 = w[3] * ca;
                    const float i0 = w[0] * cb, i1 = w[1] * cb, i2 = w[2] * cb, i3 = w[3] * cb;
                    const unsigned rh0 = pack_bf16(r0, r1), rh1 = pack_bf16(r2, r3);
                    const unsigned ih0 = pack_bf16(i0, i1), ih1 = pack_bf16(i2, i3);
                    const unsigned rl0 = pack_lo(r0, r1, rh0), rl1 = pack_lo(r2, r3, rh1);
                    const unsigned il0 = pack_lo(i0, i1, ih0), il1 = pack_lo(i2, i3, ih1);
                    u32x4 vrh, vrl, vih, vil;
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        vrh[o] = __builtin_amdgcn_perm(rh1, rh0, sel[o]);
                        vrl[o] = __builtin_amdgcn_perm(rl1, rl0, sel[o]);
                        vih[o] = __builtin_amdgcn_perm(ih1, ih0, sel[o]);
                        vil[o] = __builtin_amdgcn_perm(il1, il0, sel[o]);
                    }
                    const bf16x8 brh = __builtin_bit_cast(bf16x8, vrh), brl = __builtin_bit_cast(bf16x8, vrl);
                    const bf16x8 bih = __builtin_bit_cast(bf16x8, vih), bil = __builtin_bit_cast(bf16x8, vil);
#pragma unroll
                    for (int t = 0; t < KT; ++t) {
                        const unsigned char* p = ap + t * 16 * RB;
                        const u32x2 h0 = *reinterpret_cast<const u32x2*>(p);
                        const u32x2 h1 = *reinterpret_cast<const u32x2*>(ap + dq[0] + t * 16 * RB);
                        const u32x2 l0 = *reinterpret_cast<const u32x2*>(ap + dq[1] + t * 16 * RB);
                        const u32x2 l1 = *reinterpret_cast<const u32x2*>(ap + dq[2] + t * 16 * RB);
                        const bf16x8 vah = __builtin_bit_cast(bf16x8, u32x4{h0[0], h0[1], h1[0], h1[1]});
                        const bf16x8 val = __builtin_bit_cast(bf16x8, u32x4{l0[0], l0[1], l1[0], l1[1]});
                        accr[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, brh, accr[g][t], 0, 0, 0);
                        acci[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, bih, acci[g][t], 0, 0, 0);
                        accr[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, brl, accr[g][t], 0, 0, 0);
                        acci[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, bil, acci[g][t], 0, 0, 0);
                        accr[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(val, brh, accr[g][t], 0, 0, 0);
                        acci[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(val, bih, acci[g][t], 0, 0, 0);
                    }
                }
            }
            if (c % CPS == CPS - 1 || c + 1 == ce) {   // end of a stage (workgroup-uniform)
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
            }
        }
    }

    // D layout: lane holds column (pixel) lane & 15, rows 4 (lane / 16) + v
    const float osc = SP ? ldexpf(1.f, a.qexp[kProfileScaleParts]) : 1.f;
    if (piece >= 0) {
        // a piece's partial spectrum of the tile: [pixel ly * TX + lx][k_z
        // bin of the block], every pixel and bin (tail_combine_kernel keeps
        // those inside the image and the scan)
        float2* pp = a.part + static_cast<size_t>(piece) * (TX * TY * KB);
#pragma unroll
        for (int g = 0; g < GPW; ++g) {
            float2* out = pp + ((gpy[g] - ty0) * TX + (gpx[g] - tx0)) * KB;
#pragma unroll
            for (int t = 0; t < KT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    out[16 * t + 4 * kg + v] = make_float2(accr[g][t][v] * osc, acci[g][t][v] * osc);
        }
        return;
    }
#pragma unroll
    for (int g = 0; g < GPW; ++g) {
        if (gpx[g] < a.nx && gpy[g] < a.ny) {
            float2* out = G + (static_cast<size_t>(gpy[g]) * a.nx + gpx[g]) * a.n_z;
#pragma unroll
            for (int t = 0; t < KT; ++t) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int kz = blk * KB + 16 * t + 4 * kg + v;
                    if (kz < a.n_z) out[kz] = make_float2(accr[g][t][v] * osc, acci[g][t][v] * osc);
                }
            }
        }
    }
}

struct TailArgs {
    int n_whole, n_part, n_tiles, tiles_x, tx, ty, kb, nx, ny, n_z;
    long long n_elems;   // tail items x elements per piece
};

// Sum of the pieces' partial spectra of every split work item, in piece
// order (deterministic), into the item's pixels and k_z bins of G.
__global__ void tail_combine_kernel(const float2* __restrict__ part, TailArgs a, float2* __restrict__ G) {
    const int tp = a.tx * a.ty * a.kb;   // elements per piece
    for (long long e = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; e < a.n_elems;
         e += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int t = static_cast<int>(e / tp), r = static_cast<int>(e - static_cast<long long>(t) * tp);
        const int lp = r / a.kb, lk = r - lp * a.kb;
        const int work = a.n_whole + t;
        const int blk = work / a.n_tiles, tile = work - blk * a.n_tiles;
        const int gx = (tile % a.tiles_x) * a.tx + lp % a.tx, gy = (tile / a.tiles_x) * a.ty + lp / a.tx;
        const int kz = blk * a.kb + lk;
        if (gx >= a.nx || gy >= a.ny || kz >= a.n_z) continue;
        const float2* src = part + static_cast<size_t>(t) * a.n_part * tp + r;
        float2 acc = src[0];
        for (int k = 1; k < a.n_part; ++k) {
            const float2 v = src[static_cast<size_t>(k) * tp];
            acc.x += v.x;
            acc.y += v.y;
        }
        G[(static_cast<size_t>(gy) * a.nx + gx) * a.n_z + kz] = acc;
    }
}

// Tail split.  With S workgroups resident at once (occupancy x CUs), the
// items beyond the last full round, T = n_work mod S of them, would run as
// a round of their own with most of the GPU idle.  If T <= S / 2, each of
// them is instead split into k = min(S / T, groups of four channels, the
// workspace's pieces / T) pieces over its channels: the pieces fill that
// round with work of 1 / k of an item each and write partial spectra, which
// tail_combine_kernel adds (a second launch on the same stream).
template <int GPW, int KT, int NW, bool SP>
int launch_cfg(BpmArgs a, size_t smem, long long cap_pieces, hipStream_t s, const unsigned short* qs,
               const GatherTileEntry* tab, float2* G) {
    constexpr int NG = GPW * NW, GX = NG == 4 ? 2 : 4, TX = 4 * GX, TY = 4 * (NG / GX), KB = 16 * KT;
    auto fn = backproject_mfma_kernel<GPW, KT, NW, SP>;
    if (smem > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem));
        if (e != hipSuccess)
            return fail(PL_EDEVICE, "MFMA back-projection LDS of %zu bytes: %s", smem, hipGetErrorString(e));
    }
    static std::atomic<int> per_cu_cache{-1};   // this kernel's resident workgroups per CU
    int per_cu = per_cu_cache.load(std::memory_order_relaxed);
    if (per_cu < 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), 64 * NW, smem) !=
            hipSuccess)
            return fail(PL_EDEVICE, "MFMA back-projection: occupancy query failed");
        per_cu_cache.store(per_cu, std::memory_order_relaxed);
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(PL_EDEVICE, "MFMA back-projection: device query failed");
    const long long slots = static_cast<long long>(per_cu) * cus;
    a.n_whole = a.n_work;
    a.n_part = 1;
    if (slots > 0 && a.part) {
        const long long tail = a.n_work % slots;
        if (tail > 0 && 2 * tail <= slots) {
            const long long k = std::min({slots / tail, static_cast<long long>(a.n_ch4), cap_pieces / tail});
            if (k >= 2) {
                a.n_whole = static_cast<int>(a.n_work - tail);
                a.n_part = static_cast<int>(k);
            }
        }
    }
    a.per_xcd = (a.n_whole + 7) / 8;
    a.grid_whole = 8 * a.per_xcd;
    a.per_xcd_tail = static_cast<int>((static_cast<long long>(a.n_work - a.n_whole) * a.n_part + 7) / 8);
    const long long blocks = a.grid_whole + 8LL * a.per_xcd_tail;
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(64 * NW), smem, s, qs, tab, a, G);
    int rc = check_launch("back-projection (MFMA)");
    if (rc || a.n_part == 1) return rc;
    TailArgs t{};
    t.n_whole = a.n_whole;
    t.n_part = a.n_part;
    t.n_tiles = a.n_tiles;
    t.tiles_x = a.tiles_x;
    t.tx = TX;
    t.ty = TY;
    t.kb = KB;
    t.nx = a.nx;
    t.ny = a.ny;
    t.n_z = a.n_z;
    t.n_elems = static_cast<long long>(a.n_work - a.n_whole) * TX * TY * KB;
    const unsigned cblocks = static_cast<unsigned>(std::min<long long>((t.n_elems + 255) / 256, 8192));
    hipLaunchKernelGGL(tail_combine_kernel, dim3(cblocks), dim3(256), 0, s, a.part, t, G);
    return check_launch("back-projection (MFMA) tail combine");
}

}  // namespace

size_t backproject_mfma_lds_bytes(int kz_block, bool single_pass) {
    return kSelEntries * 16 + 2ull * stage_channels(single_pass, kz_block) * kz_block * 16 * row_chunks(single_pass);
}

size_t backproject_mfma_part_bytes(const HybridPlan& p) {
    if (!p.bp_mfma) return 0;
    const long long items = static_cast<long long>(p.tiles_x) * p.tiles_y * p.n_blocks;
    const long long pieces = std::min<long long>(kMaxTailPieces, items * ((p.n_ch + 3) / 4));
    return static_cast<size_t>(pieces) * p.tile_x * p.tile_y * p.block * sizeof(float2);
}

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
    a.n_ch4 = (p.n_ch + 3) / 4;
    a.part = reinterpret_cast<float2*>(ws + p.off_part);
    a.nck = p.window / 8;
    a.mono = p.mode == PL_MONO;
    a.qexp = reinterpret_cast<const int*>(ws + p.off_qexp);
    a.x0 = p.x0;
    a.y0 = p.y0;
    a.dx = p.dx;
    a.dy = p.dy;
    a.inv_du = 1.0 / p.du;
    std::memcpy(a.coef, p.coef, sizeof(a.coef));
    for (int b = 0; b < kMaxBlocks; ++b) a.kref[b] = p.kref[b];
    if (p.window % 8 || a.nck < 2 || a.nck > 8 || p.window > p.n_l || p.window_pad != row_chunks(p.bp_mfma_sp))
        return fail(PL_EUNSUPPORTED, "MFMA back-projection window %d out of range", p.window);
    const size_t smem = backproject_mfma_lds_bytes(p.block, p.bp_mfma_sp);
    if (smem > kMaxLds) return fail(PL_EUNSUPPORTED, "MFMA back-projection needs %zu bytes of LDS", smem);
    const GatherTileEntry* tab = reinterpret_cast<const GatherTileEntry*>(ws + p.off_tiles);
    (void)dt;
    const long long cap_pieces =
        static_cast<long long>(backproject_mfma_part_bytes(p) / (static_cast<size_t>(p.tile_x) * p.tile_y * p.block * sizeof(float2)));
    const int ng = p.tile_x * p.tile_y / 16;
    const int kt = p.block / 16;
    const int nw = p.waves;
#define PL_BPM(G_, K_, W_)                                                                              \
    if (ng == G_ * W_ && kt == K_ && nw == W_)                                                          \
        return p.bp_mfma_sp ? launch_cfg<G_, K_, W_, true>(a, smem, cap_pieces, s, qs, tab, G)           \
                            : launch_cfg<G_, K_, W_, false>(a, smem, cap_pieces, s, qs, tab, G);
    PL_BPM(1, 4, 4) PL_BPM(1, 8, 4) PL_BPM(2, 4, 4) PL_BPM(2, 8, 4) PL_BPM(4, 4, 4) PL_BPM(4, 8, 4)
    PL_BPM(1, 4, 8) PL_BPM(1, 8, 8) PL_BPM(2, 4, 8)
#undef PL_BPM
    return fail(PL_EUNSUPPORTED, "MFMA back-projection tile %dx%d with %d k_z bins and %d wavefronts", p.tile_x,
                p.tile_y, p.block, p.waves);
}

#undef PL_STAGE_ROWS
#undef PL_DMA16

}  // namespace pl
