// Adjoint of the range compression (the type-2 transform of eq. 8a / 19a):
//   S~[c][kz][f] = w[kz][f] sum_i q~[c][kz][i] exp(-j k'[kz][f] (l_lo[c] + i du)),
// the transpose of q[c][kz][i] = sum_f w[kz][f] S[c][kz][f] exp(+j k' l_i),
// which the forward path evaluates by NUFFT.  Here the sums are direct: one
// wavefront per (c, kz), lanes over frequencies, the profile read 64 samples
// per coalesced load and broadcast by readlane, the phasor advanced by a
// recurrence in FP32 and re-anchored from an FP64-reduced phase every 32
// samples.
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

}  // namespace

int launch_range_adjoint(const HybridPlan& p, const float2* qt, char* ws, float2* St, hipStream_t s) {
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
