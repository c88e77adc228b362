// Range compression, eq. (8a) / (19a), as a dense contraction on the matrix
// cores.  For one k_z bin the range profiles of all channels are
//   Q[i][c] = sum_f A[i][f] C[f][c],  A[i][f] = exp(j k'_f u_i),
//   C[f][c] = w_f S[c][kz][f] exp(j k'_f l_mid[c]),  u_i = (i - n_l/2) du,
// i.e. the direct nonuniform DFT the NUFFT approximates, cast as a complex
// GEMM with M = n_l, N = n_ch, K = n_f.  Complex products use the real
// embedding with one phasor operand A' = [Re A | -Im A] (K' = 2 n_f):
//   Re Q = A' [Re C; Im C],   Im Q = A' [Im C; -Re C].
// Operands are BF16 or FP16 split into hi + lo parts (x = hi + lo, each
// rounded to nearest), and each product is hi*hi + hi*lo + lo*hi with FP32
// accumulation in the matrix cores (v_mfma_f32_32x32x16_{bf16,f16} on
// 32-row wavefronts below 64 frequencies, v_mfma_f32_16x16x32 on 16-row
// wavefronts from 64 up, where the phasor operand's registers would
// otherwise leave one or two wavefronts per SIMD).  The
// phasor phase k'_f u_i is formed in float64 and range-reduced before the
// float32 sin/cos.  FP16 strengths carry a power-of-2 scale per (k_z,
// channel) so their largest part sits near 2^14.
//
// Output forms: complex64 profiles; four BF16 planes per (channel, k_z) (Re
// hi, Re lo, Im hi, Im lo) for the split matrix-core back-projection; or two
// FP16 planes (Re, Im) times one power of two 2^-g for the whole call, for
// its single-pass form.  With m(k_z, c) the largest |Re|, |Im| of the
// strengths of a pair, |Re Q|, |Im Q| <= 2 n_f m (the phasors have modulus 1),
// so g = ceil(log2 n_f) + 1 + max log2-exponent of m - 14 keeps every FP16
// value below 2^15 whatever the data; FP16's exponent range leaves values
// down to 2^-29 of that bound at full relative precision.
#include "device.hpp"

namespace pl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool F16>
struct Half;
template <>
struct Half<false> {
    typedef __bf16 T;
    typedef bf16x8 V;
    static __device__ __forceinline__ f32x16 mfma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ f32x4 mfma16(V a, V b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Half<true> {
    typedef _Float16 T;
    typedef f16x8 V;
    static __device__ __forceinline__ f32x16 mfma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ f32x4 mfma16(V a, V b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

struct MfmaArgs {
    int n_ch, n_chp, n_z, n_f, n_fp, n_l;
    double du;
};

// Strengths C[f][c] of one channel and kStrengthBins consecutive k_z bins
// per wavefront (every load of the bins issued before the arithmetic),
// split into hi / lo parts of Re and Im: cs[((kz * n_chp + c) * 4 + part) *
// n_fp + f], part 0 Re hi, 1 Re lo, 2 Im hi, 3 Im lo; padded frequencies and
// channels are zero.  se[kz * n_chp + c] is the power-of-2 scale exponent.
constexpr int kStrengthBins = 4;
template <bool F16>
__global__ __launch_bounds__(256) void strengths_kernel(const float2* __restrict__ spec,
                                                        const double* __restrict__ llo,
                                                        const double* __restrict__ kp,
                                                        const float* __restrict__ wk, MfmaArgs a,
                                                        typename Half<F16>::T* __restrict__ cs,
                                                        int* __restrict__ se) {
    typedef typename Half<F16>::T T;
    constexpr int KB = kStrengthBins;
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int n_groups = (a.n_z + KB - 1) / KB;
    if (wid >= n_groups * a.n_chp) return;
    const int kap0 = (wid / a.n_chp) * KB, c = wid % a.n_chp;
    float2 s[KB][2], v[KB][2];
    double kpf[KB][2];
    float w[KB][2];
    const bool chan = c < a.n_ch;
    const double lmid = chan ? llo[c] + (a.n_l / 2) * a.du : 0.0;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        const int kap = kap0 + j;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int f = lane + 64 * h;   // n_fp <= 128
            s[j][h] = make_float2(0.f, 0.f);
            kpf[j][h] = 0.0;
            w[j][h] = 0.f;
            if (chan && kap < a.n_z && f < a.n_f) {
                const size_t e = static_cast<size_t>(kap) * a.n_f + f;
                s[j][h] = spec[(static_cast<size_t>(c) * a.n_z + kap) * a.n_f + f];
                kpf[j][h] = kp[e];
                w[j][h] = wk[e];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        const int kap = kap0 + j;
        if (kap >= a.n_z) break;   // wavefront-uniform
        float mx = 0.f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            v[j][h] = cscale(cmul(s[j][h], cis(kpf[j][h] * lmid)), w[j][h]);
            mx = fmaxf(mx, fmaxf(fabsf(v[j][h].x), fabsf(v[j][h].y)));
        }
        int ex = 0;
        if (F16) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
            // all-zero pairs (padding, evanescent k_z) take the largest
            // exponent, so they never decide the single-pass scale below
            ex = mx > 0.f ? min(max(14 - ilogbf(mx), -100), 100) : 100;
        }
        const float sc = ldexpf(1.f, ex);
        T* dst = cs + (static_cast<size_t>(kap) * a.n_chp + c) * 4 * a.n_fp;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int f = lane + 64 * h;
            if (f < a.n_fp) {
                const float re = v[j][h].x * sc, im = v[j][h].y * sc;
                const T rh = static_cast<T>(re), ih = static_cast<T>(im);
                dst[f] = rh;
                dst[a.n_fp + f] = static_cast<T>(re - static_cast<float>(rh));
                dst[2 * a.n_fp + f] = ih;
                dst[3 * a.n_fp + f] = static_cast<T>(im - static_cast<float>(ih));
            }
        }
        if (lane == 0) se[static_cast<size_t>(kap) * a.n_chp + c] = ex;
    }
}

__device__ __forceinline__ u32x4 neg16(u32x4 x) { return x ^ 0x80008000u; }

// Scale exponent g of the single-pass FP16 profiles (see the header), in
// two steps: kProfileScaleParts workgroups each take the smallest strength
// exponent of their share of (k_z, channel) into part[b]; every workgroup of
// the contraction then reduces the parts itself (one load per lane) and the
// first one stores g for the back-projection in part[kProfileScaleParts].
__global__ __launch_bounds__(256) void profile_scale_kernel(const int* __restrict__ se, int n, int* __restrict__ part) {
    __shared__ int wmin[4];
    const int per = (n + kProfileScaleParts - 1) / kProfileScaleParts;
    const int lo = blockIdx.x * per, hi = min(n, lo + per);
    int m = 100;
    for (int i = lo + threadIdx.x; i < hi; i += 256) m = min(m, se[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
}

__device__ __forceinline__ int profile_scale(const int* __restrict__ part, int log2_nf) {
    int m = (threadIdx.x & 63) < kProfileScaleParts ? part[threadIdx.x & 63] : 100;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o));
    return log2_nf + 1 - m;
}

__device__ __forceinline__ unsigned short bf16_of(float x) {
    return __builtin_bit_cast(unsigned short, static_cast<__bf16>(x));
}

// 16-byte direct global-to-LDS copy (device pass only; the host pass of
// this translation unit emits the launch stubs and must not see it).
#if defined(__HIP_DEVICE_COMPILE__)
#define PL_DMA16(SRC, DST) __builtin_amdgcn_global_load_lds((SRC), (DST), 16, 0, 0)
#else
#define PL_DMA16(SRC, DST) ((void)(SRC), (void)(DST))
#endif

// LDS bytes of range_mfma_kernel: two buffers of one channel tile's
// strengths (32 channels x 4 parts x n_fp values).
__host__ __device__ constexpr int range_mfma_lds(int n_fp) { return 2 * 32 * 4 * n_fp * 2; }

// One block = one k_z bin x 128 range samples; wavefront w owns rows
// [32 w, 32 w + 32) of that range block and keeps its phasor operand A' for
// all of K' in registers, then walks the channel tiles of 32.  The four
// wavefronts share each tile's strengths: the block copies them into LDS
// (16-byte direct copies, one tile ahead, double-buffered; chunk j of
// channel c at position j ^ (c & 15) of the channel's row, c & 7 when the
// row has an odd multiple of 8 chunks, so that the lanes of consecutive
// channels read distinct banks).  The blocks of one k_z bin run
// on one XCD (block b runs on XCD b mod 8): the bin's strengths come from
// memory into that XCD's L2 once.
// OUT: kOutC64 complex64 profiles; kOutSplit four BF16 planes per
// (channel, k_z) -- Re hi, Re lo, Im hi, Im lo with x = hi + lo -- the
// operand layout of the split matrix-core back-projection; kOutF16 two FP16
// planes (Re, Im) scaled by 2^-g, that of its single-pass form (g from the
// exponent parts in qexp[0, kProfileScaleParts), stored to
// qexp[kProfileScaleParts]).
constexpr int kOutC64 = 0, kOutSplit = 1, kOutF16 = 2;
template <bool F16, int NCH, int OUT>
__global__ __launch_bounds__(256) void range_mfma_kernel(const typename Half<F16>::T* __restrict__ cs,
                                                         const int* __restrict__ se,
                                                         const double* __restrict__ kp, MfmaArgs a,
                                                         int* __restrict__ qexp, int log2_nf, void* __restrict__ qout) {
    typedef typename Half<F16>::T T;
    typedef typename Half<F16>::V V;
    constexpr int NC = NCH;          // chunks of 16 in K' = 2 n_fp, NC = n_fp / 8
    constexpr int HC = NC / 2;       // chunks per half (Re part / Im part)
    constexpr int NFP = 8 * NCH;     // padded frequencies (a.n_fp)
    constexpr int CPC = NFP / 2;     // 16-byte chunks per channel (4 parts)
    constexpr int SWZ = CPC % 16 == 0 ? 15 : 7;
    constexpr int NDMA = 32 * CPC / 256;   // copies per thread and tile
    static_assert(32 * CPC % 256 == 0, "a tile is a whole number of block-wide copies");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int n_ib = (a.n_l + 127) / 128;
    const int slot = blockIdx.x >> 3;
    const int kap = (slot / n_ib) * 8 + (blockIdx.x & 7);
    const int ib = slot % n_ib;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = ib * 128 + wave * 32;
    int gexp = 0;
    if constexpr (OUT == kOutF16) {
        gexp = profile_scale(qexp, log2_nf);
        if (blockIdx.x == 0 && threadIdx.x == 0) qexp[kProfileScaleParts] = gexp;
    }
    if (kap >= a.n_z) return;   // the whole block, before any barrier
    const bool active = row0 < a.n_l;   // wavefronts past n_l only copy
    const int n_ct = a.n_chp / 32;

    // copies of tile ct into buffer ct & 1: thread t's j-th copy fills LDS
    // chunk p = (4 j + wave) * 64 + lane, channel p / CPC, swizzled chunk
    // p % CPC, from the channel's chunk (p % CPC) ^ (channel & SWZ)
    const char* tile0 = reinterpret_cast<const char*>(cs + static_cast<size_t>(kap) * a.n_chp * 4 * NFP);
    unsigned soff[NDMA];
#pragma unroll
    for (int j = 0; j < NDMA; ++j) {
        const int pch = (4 * j + wave) * 64 + lane;
        const int ch = pch / CPC, js = pch - ch * CPC;
        soff[j] = static_cast<unsigned>((ch * CPC + (js ^ (ch & SWZ))) * 16);
    }
    auto stage = [&](int ct) {
        const char* src = tile0 + static_cast<size_t>(ct) * 32 * CPC * 16;
        unsigned char* dst = smem + (ct & 1) * (32 * CPC * 16);
#pragma unroll
        for (int j = 0; j < NDMA; ++j) PL_DMA16(src + soff[j], dst + (4 * j + wave) * 1024);
    };
    stage(0);
    const int i = row0 + (lane & 31);
    const int kh = 8 * (lane >> 5);  // this lane's k' offset inside a chunk

    // phasor operand: chunk q < HC holds Re A at f = 16 q + kh + t, chunk
    // q + HC holds -Im A at the same f
    V ah[NC], al[NC];
    {
        const double u = (i - a.n_l / 2) * a.du;
        const bool row_ok = i < a.n_l;
#pragma unroll
        for (int qq = 0; qq < HC; ++qq) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int f = 16 * qq + kh + t;
                float cr = 0.f, ci = 0.f;
                if (row_ok && f < a.n_f) {
                    const float2 e = cis(kp[static_cast<size_t>(kap) * a.n_f + f] * u);
                    cr = e.x;
                    ci = -e.y;
                }
                const T crh = static_cast<T>(cr), cih = static_cast<T>(ci);
                ah[qq][t] = crh;
                al[qq][t] = static_cast<T>(cr - static_cast<float>(crh));
                ah[qq + HC][t] = cih;
                al[qq + HC][t] = static_cast<T>(ci - static_cast<float>(cih));
            }
        }
    }

    const int cl = lane & 31;   // this lane's channel in the tile
    for (int ct = 0; ct < n_ct; ++ct) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();   // tile ct in LDS; every wavefront done with tile ct - 1
        if (ct + 1 < n_ct) stage(ct + 1);
        if (!active) continue;
        const int c = ct * 32 + cl;
        const u32x4* base = reinterpret_cast<const u32x4*>(smem + (ct & 1) * (32 * CPC * 16)) + cl * CPC;
        constexpr int stride4 = NFP / 8;  // chunks per part
        f32x16 accr = {}, acci = {};
#pragma unroll
        for (int qq = 0; qq < NC; ++qq) {
            const bool second = qq >= HC;
            const int f0 = 16 * (second ? qq - HC : qq) + kh;
            const int sw = cl & SWZ;
            const u32x4 rh = base[(0 * stride4 + f0 / 8) ^ sw], rl = base[(1 * stride4 + f0 / 8) ^ sw];
            const u32x4 ih = base[(2 * stride4 + f0 / 8) ^ sw], il = base[(3 * stride4 + f0 / 8) ^ sw];
            // Re Q: B' = [Re C; Im C];  Im Q: B'' = [Im C; -Re C]
            const u32x4 b1h = second ? ih : rh, b1l = second ? il : rl;
            const u32x4 b2h = second ? neg16(rh) : ih, b2l = second ? neg16(rl) : il;
            const V vb1h = __builtin_bit_cast(V, b1h), vb1l = __builtin_bit_cast(V, b1l);
            const V vb2h = __builtin_bit_cast(V, b2h), vb2l = __builtin_bit_cast(V, b2l);
            accr = Half<F16>::mfma(ah[qq], vb1h, accr);
            accr = Half<F16>::mfma(ah[qq], vb1l, accr);
            accr = Half<F16>::mfma(al[qq], vb1h, accr);
            acci = Half<F16>::mfma(ah[qq], vb2h, acci);
            acci = Half<F16>::mfma(ah[qq], vb2l, acci);
            acci = Half<F16>::mfma(al[qq], vb2h, acci);
        }
        if (c < a.n_ch) {
            const int ex = se[static_cast<size_t>(kap) * a.n_chp + c];
            if constexpr (OUT == kOutF16) {
                const float sc = ldexpf(1.f, -ex - gexp);
                _Float16* dst = static_cast<_Float16*>(qout) + (static_cast<size_t>(c) * a.n_z + kap) * 2 * a.n_l;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int r = row0 + 8 * g + 4 * (lane >> 5);
                    if (r < a.n_l) {
                        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
                        h4 vr, vi;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            vr[k] = static_cast<_Float16>(accr[4 * g + k] * sc);
                            vi[k] = static_cast<_Float16>(acci[4 * g + k] * sc);
                        }
                        *reinterpret_cast<h4*>(dst + r) = vr;
                        *reinterpret_cast<h4*>(dst + a.n_l + r) = vi;
                    }
                }
                continue;
            }
            const float sc = ldexpf(1.f, -ex);
            if constexpr (OUT == kOutSplit) {
                // four consecutive rows per lane and plane: one 8-byte store
                // each (n_l is a multiple of 4)
                unsigned short* dst =
                    static_cast<unsigned short*>(qout) + (static_cast<size_t>(c) * a.n_z + kap) * 4 * a.n_l;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int r = row0 + 8 * g + 4 * (lane >> 5);
                    if (r < a.n_l) {
                        unsigned short rh[4], rl[4], ih[4], il[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const float xr = accr[4 * g + k] * sc, xi = acci[4 * g + k] * sc;
                            rh[k] = bf16_of(xr);
                            ih[k] = bf16_of(xi);
                            rl[k] = bf16_of(xr - __uint_as_float(static_cast<unsigned>(rh[k]) << 16));
                            il[k] = bf16_of(xi - __uint_as_float(static_cast<unsigned>(ih[k]) << 16));
                        }
                        auto pack = [](const unsigned short (&h)[4]) {
                            return make_uint2(h[0] | (static_cast<unsigned>(h[1]) << 16),
                                              h[2] | (static_cast<unsigned>(h[3]) << 16));
                        };
                        *reinterpret_cast<uint2*>(dst + r) = pack(rh);
                        *reinterpret_cast<uint2*>(dst + a.n_l + r) = pack(rl);
                        *reinterpret_cast<uint2*>(dst + 2 * a.n_l + r) = pack(ih);
                        *reinterpret_cast<uint2*>(dst + 3 * a.n_l + r) = pack(il);
                    }
                }
            } else {
                float2* dst = static_cast<float2*>(qout) + (static_cast<size_t>(c) * a.n_z + kap) * a.n_l;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int r = row0 + 8 * (v / 4) + 4 * (lane >> 5) + (v & 3);
                    if (r < a.n_l) dst[r] = make_float2(accr[v] * sc, acci[v] * sc);
                }
            }
        }
    }
}

// The same contraction for 64 or more frequencies, where the 32-row
// form's phasor registers leave one or two wavefronts per SIMD: a wavefront
// owns 16 rows (v_mfma_f32_16x16x32: lane l holds row or column l & 15 and
// K' values 8 (l / 16) .. + 7 of a chunk of 32; the result rows 4 (l / 16)
// .. + 3 of column l & 15), a block of four wavefronts 64 rows, and the
// channel tiles are 16 wide, staged in LDS as in range_mfma_kernel.
constexpr int kRows16 = 64;
__host__ __device__ constexpr int range_mfma16_lds(int n_fp) { return 2 * 16 * 4 * n_fp * 2; }
template <bool F16, int NCH, int OUT>
__global__ __launch_bounds__(256) void range_mfma16_kernel(const typename Half<F16>::T* __restrict__ cs,
                                                           const int* __restrict__ se,
                                                           const double* __restrict__ kp, MfmaArgs a,
                                                           int* __restrict__ qexp, int log2_nf,
                                                           void* __restrict__ qout) {
    typedef typename Half<F16>::T T;
    typedef typename Half<F16>::V V;
    constexpr int NFP = 8 * NCH;          // padded frequencies (a.n_fp)
    constexpr int NQ = NCH / 2;           // chunks of 32 in K' = 2 n_fp
    constexpr int CPC = NFP / 2;          // 16-byte chunks per channel (4 parts)
    constexpr int SWZ = CPC % 16 == 0 ? 15 : 7;
    constexpr int TILE = 16 * CPC;        // chunks per channel tile
    constexpr int NDMA = (TILE + 255) / 256;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int n_ib = (a.n_l + kRows16 - 1) / kRows16;
    const int slot = blockIdx.x >> 3;
    const int kap = (slot / n_ib) * 8 + (blockIdx.x & 7);
    const int ib = slot % n_ib;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = ib * kRows16 + wave * 16;
    int gexp = 0;
    if constexpr (OUT == kOutF16) {
        gexp = profile_scale(qexp, log2_nf);
        if (blockIdx.x == 0 && threadIdx.x == 0) qexp[kProfileScaleParts] = gexp;
    }
    if (kap >= a.n_z) return;   // the whole block, before any barrier
    const bool active = row0 < a.n_l;
    const int n_ct = a.n_chp / 16;

    // copies of tile ct into buffer ct & 1: thread t's j-th copy fills LDS
    // chunk p = (4 j + wave) * 64 + lane (lanes past the tile idle)
    const char* tile0 = reinterpret_cast<const char*>(cs + static_cast<size_t>(kap) * a.n_chp * 4 * NFP);
    unsigned soff[NDMA];
#pragma unroll
    for (int j = 0; j < NDMA; ++j) {
        const int pch = (4 * j + wave) * 64 + lane;
        const int ch = pch / CPC, js = pch - ch * CPC;
        soff[j] = pch < TILE ? static_cast<unsigned>((ch * CPC + (js ^ (ch & SWZ))) * 16) : ~0u;
    }
    auto stage = [&](int ct) {
        const char* src = tile0 + static_cast<size_t>(ct) * TILE * 16;
        unsigned char* dst = smem + (ct & 1) * (TILE * 16);
#pragma unroll
        for (int j = 0; j < NDMA; ++j)
            if ((4 * j + wave) * 64 < TILE && soff[j] != ~0u) PL_DMA16(src + soff[j], dst + (4 * j + wave) * 1024);
    };
    stage(0);
    const int i = row0 + (lane & 15);
    const int kh = 8 * (lane >> 4);   // this lane's k' offset inside a chunk

    // phasor operand: the lane's 8 values of chunk q are k' = 32 q + kh + t;
    // k' < n_fp holds Re A at f = k', k' >= n_fp holds -Im A at f = k' - n_fp
    V ah[NQ], al[NQ];
    {
        const double u = (i - a.n_l / 2) * a.du;
        const bool row_ok = i < a.n_l;
        const double* kprow = kp + static_cast<size_t>(kap) * a.n_f;
        auto put = [&](int q, int t, float x) {
            const T xh = static_cast<T>(x);
            ah[q][t] = xh;
            al[q][t] = static_cast<T>(x - static_cast<float>(xh));
        };
        if constexpr (NFP % 32 == 0) {
            // chunk q + NQ / 2 holds -Im A at the frequencies of chunk q
#pragma unroll
            for (int q = 0; q < NQ / 2; ++q) {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int f = 32 * q + kh + t;
                    float2 e = make_float2(0.f, 0.f);
                    if (row_ok && f < a.n_f) e = cis(kprow[f] * u);
                    put(q, t, e.x);
                    put(q + NQ / 2, t, -e.y);
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int k0 = 32 * q + kh;
                const bool im = k0 >= NFP;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int f = (im ? k0 - NFP : k0) + t;
                    float2 e = make_float2(0.f, 0.f);
                    if (row_ok && f < a.n_f) e = cis(kprow[f] * u);
                    put(q, t, im ? -e.y : e.x);
                }
            }
        }
    }

    const int cl = lane & 15;   // this lane's channel in the tile
    for (int ct = 0; ct < n_ct; ++ct) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();   // tile ct in LDS; every wavefront done with tile ct - 1
        if (ct + 1 < n_ct) stage(ct + 1);
        if (!active) continue;
        const int c = ct * 16 + cl;
        const u32x4* base = reinterpret_cast<const u32x4*>(smem + (ct & 1) * (TILE * 16)) + cl * CPC;
        constexpr int stride4 = NFP / 8;   // chunks per part
        const int sw = cl & SWZ;
        f32x4 accr = {}, acci = {};
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int k0 = 32 * q + kh;
            const bool second = k0 >= NFP;
            const int f0 = second ? k0 - NFP : k0;
            const u32x4 rh = base[(0 * stride4 + f0 / 8) ^ sw], rl = base[(1 * stride4 + f0 / 8) ^ sw];
            const u32x4 ih = base[(2 * stride4 + f0 / 8) ^ sw], il = base[(3 * stride4 + f0 / 8) ^ sw];
            // Re Q: B' = [Re C; Im C];  Im Q: B'' = [Im C; -Re C]
            const u32x4 b1h = second ? ih : rh, b1l = second ? il : rl;
            const u32x4 b2h = second ? neg16(rh) : ih, b2l = second ? neg16(rl) : il;
            const V vb1h = __builtin_bit_cast(V, b1h), vb1l = __builtin_bit_cast(V, b1l);
            const V vb2h = __builtin_bit_cast(V, b2h), vb2l = __builtin_bit_cast(V, b2l);
            accr = Half<F16>::mfma16(ah[q], vb1h, accr);
            accr = Half<F16>::mfma16(ah[q], vb1l, accr);
            accr = Half<F16>::mfma16(al[q], vb1h, accr);
            acci = Half<F16>::mfma16(ah[q], vb2h, acci);
            acci = Half<F16>::mfma16(ah[q], vb2l, acci);
            acci = Half<F16>::mfma16(al[q], vb2h, acci);
        }
        if (c >= a.n_ch) continue;
        const int ex = se[static_cast<size_t>(kap) * a.n_chp + c];
        const int r = row0 + 4 * (lane >> 4);   // rows r .. r + 3 of column c
        if constexpr (OUT == kOutF16) {
            // n_l is a multiple of 4: the four rows are all in range or all out
            if (r < a.n_l) {
                const float sc = ldexpf(1.f, -ex - gexp);
                _Float16* dst = static_cast<_Float16*>(qout) + (static_cast<size_t>(c) * a.n_z + kap) * 2 * a.n_l;
                typedef _Float16 h4 __attribute__((ext_vector_type(4)));
                h4 vr, vi;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    vr[k] = static_cast<_Float16>(accr[k] * sc);
                    vi[k] = static_cast<_Float16>(acci[k] * sc);
                }
                *reinterpret_cast<h4*>(dst + r) = vr;
                *reinterpret_cast<h4*>(dst + a.n_l + r) = vi;
            }
        } else if constexpr (OUT == kOutSplit) {
            if (r < a.n_l) {
                const float sc = ldexpf(1.f, -ex);
                unsigned short* dst =
                    static_cast<unsigned short*>(qout) + (static_cast<size_t>(c) * a.n_z + kap) * 4 * a.n_l;
                unsigned short rh[4], rl[4], ih[4], il[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float xr = accr[k] * sc, xi = acci[k] * sc;
                    rh[k] = bf16_of(xr);
                    ih[k] = bf16_of(xi);
                    rl[k] = bf16_of(xr - __uint_as_float(static_cast<unsigned>(rh[k]) << 16));
                    il[k] = bf16_of(xi - __uint_as_float(static_cast<unsigned>(ih[k]) << 16));
                }
                auto pack = [](const unsigned short (&h)[4]) {
                    return make_uint2(h[0] | (static_cast<unsigned>(h[1]) << 16),
                                      h[2] | (static_cast<unsigned>(h[3]) << 16));
                };
                *reinterpret_cast<uint2*>(dst + r) = pack(rh);
                *reinterpret_cast<uint2*>(dst + a.n_l + r) = pack(rl);
                *reinterpret_cast<uint2*>(dst + 2 * a.n_l + r) = pack(ih);
                *reinterpret_cast<uint2*>(dst + 3 * a.n_l + r) = pack(il);
            }
        } else {
            const float sc = ldexpf(1.f, -ex);
            float2* dst = static_cast<float2*>(qout) + (static_cast<size_t>(c) * a.n_z + kap) * a.n_l;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (r + k < a.n_l) dst[r + k] = make_float2(accr[k] * sc, acci[k] * sc);
        }
    }
}

template <bool F16, int OUT>
int run_mfma(const HybridPlan& p, const float2* spec, char* ws, void* q, hipStream_t s) {
    typedef typename Half<F16>::T T;
    MfmaArgs a{};
    a.n_ch = p.n_ch;
    a.n_chp = p.n_chp;
    a.n_z = p.n_z;
    a.n_f = p.n_f;
    a.n_fp = p.n_fp;
    a.n_l = p.n_l;
    a.du = p.du;
    T* cs = reinterpret_cast<T*>(ws + p.off_mfma_b);
    int* se = reinterpret_cast<int*>(ws + p.off_mfma_a);
    const long long waves = static_cast<long long>(p.n_z) * p.n_chp;   // (k_z, channel) pairs
    const long long swaves = static_cast<long long>((p.n_z + kStrengthBins - 1) / kStrengthBins) * p.n_chp;
    hipLaunchKernelGGL(strengths_kernel<F16>, dim3(static_cast<unsigned>((swaves + 3) / 4)), dim3(256), 0, s, spec,
                       reinterpret_cast<const double*>(ws + p.off_llo), reinterpret_cast<const double*>(ws + p.off_kp),
                       reinterpret_cast<const float*>(ws + p.off_wk), a, cs, se);
    int rc = check_launch("range compression (strengths)");
    if (rc) return rc;
    int* qexp = reinterpret_cast<int*>(ws + p.off_qexp);
    int log2_nf = 0;
    while ((1 << log2_nf) < p.n_f) ++log2_nf;
    if (OUT == kOutF16) {
        hipLaunchKernelGGL(profile_scale_kernel, dim3(kProfileScaleParts), dim3(256), 0, s, se, static_cast<int>(waves), qexp);
        if ((rc = check_launch("range compression (profile scale)"))) return rc;
    }
    // the blocks of k_z bin kap are (j * n_ib + ib) * 8 + kap % 8 with
    // j = kap / 8: all on one XCD
    const long long blocks = 8LL * ((p.n_z + 7) / 8) * ((p.n_l + 127) / 128);
    const int lds = range_mfma_lds(p.n_fp);
    const double* kp = reinterpret_cast<const double*>(ws + p.off_kp);
    // 64 or more frequencies: 16-row wavefronts (the 32-row form's phasor
    // registers leave two wavefronts per SIMD at 64 and one at 128; the
    // 16-row form keeps three to five)
    const long long blocks16 = 8LL * ((p.n_z + 7) / 8) * ((p.n_l + kRows16 - 1) / kRows16);
    const int lds16 = range_mfma16_lds(p.n_fp);
    switch (p.n_fp / 8) {
#define PL_NC(N)                                                                                          \
    case N:                                                                                               \
        hipLaunchKernelGGL((range_mfma_kernel<F16, N, OUT>), dim3(static_cast<unsigned>(blocks)), dim3(256), lds, s, cs, se, \
                           kp, a, qexp, log2_nf, q);                                                      \
        break;
#define PL_NC16(N)                                                                                        \
    case N:                                                                                               \
        hipLaunchKernelGGL((range_mfma16_kernel<F16, N, OUT>), dim3(static_cast<unsigned>(blocks16)), dim3(256), lds16, s, \
                           cs, se, kp, a, qexp, log2_nf, q);                                              \
        break;
        PL_NC(2) PL_NC(4) PL_NC(6) PL_NC16(8) PL_NC16(10) PL_NC16(12) PL_NC16(14) PL_NC16(16)
#undef PL_NC
#undef PL_NC16
        default:
            return fail(PL_EUNSUPPORTED, "MFMA range compression supports up to 128 frequencies");
    }
    return check_launch("range compression (MFMA)");
}

}  // namespace

int launch_range_compress_mfma(const HybridPlan& p, const float2* spec, char* ws, float2* q, hipStream_t s) {
    if (p.n_fp > 128 || p.n_fp % 16 != 0) return fail(PL_EUNSUPPORTED, "MFMA range compression supports up to 128 frequencies");
    return p.precision == PL_PREC_FP16 ? run_mfma<true, kOutC64>(p, spec, ws, q, s)
                                       : run_mfma<false, kOutC64>(p, spec, ws, q, s);
}

int launch_range_compress_mfma_split(const HybridPlan& p, const float2* spec, char* ws, unsigned short* qs,
                                     hipStream_t s) {
    if (p.n_fp > 128 || p.n_fp % 16 != 0) return fail(PL_EUNSUPPORTED, "MFMA range compression supports up to 128 frequencies");
    if (p.n_l % 4) return fail(PL_EUNSUPPORTED, "split range profiles need n_l divisible by 4");
    if (p.bp_mfma_sp) {
        if (p.precision != PL_PREC_FP16) return fail(PL_EUNSUPPORTED, "single-pass profiles are FP16");
        return run_mfma<true, kOutF16>(p, spec, ws, qs, s);
    }
    return p.precision == PL_PREC_FP16 ? run_mfma<true, kOutSplit>(p, spec, ws, qs, s)
                                       : run_mfma<false, kOutSplit>(p, spec, ws, qs, s);
}

}  // namespace pl
