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


}  // namespace pl
