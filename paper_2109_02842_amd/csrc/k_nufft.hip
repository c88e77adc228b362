// Range compression, eq. (8a) / (19a), as a type-1 NUFFT in FP32: the k'
// samples of one (channel, k_z) pair are spread onto a 2x fine grid with the
// exponential-of-semicircle kernel, transformed by an inverse FFT in LDS and
// deapodised onto the uniform range grid.
#include "device.hpp"

namespace pl {
namespace {

struct NufftArgs {
    int n_ch, n_z, n_f, n_l, n_fine;
    int pad_;
    double du, h, beta, inv_h;
    Radices rad;
};

// One block per (channel c, k_z bin kap).  With l_i = l_lo[c] + i du and the
// centre l_mid = l_lo[c] + (n_l/2) du, the strengths
//   a_f = w_f S[c][kap][f] exp(j k'_f l_mid)
// give q[i] = sum_f a_f exp(j k'_f du (i - n_l/2)) = sum_f w_f S exp(j k'_f l_i).
// The points y_f = k'_f du n_fine / (2 pi) (fine-grid cells) are sorted in f
// (k_rho grows with k; evanescent entries sit below all others and carry zero
// weight), so each fine cell gathers its neighbours by binary search: no
// atomics, deterministic.
__global__ __launch_bounds__(256) void nufft_kernel(const float2* __restrict__ spec,
                                                    const double* __restrict__ llo,
                                                    const double* __restrict__ kp,
                                                    const float* __restrict__ wk,
                                                    const float2* __restrict__ tw,
                                                    const float* __restrict__ deap, NufftArgs a,
                                                    float2* __restrict__ q) {
    extern __shared__ double smem_d[];
    double* py = smem_d;                                    // n_f fine-grid positions
    float2* pa = reinterpret_cast<float2*>(py + a.n_f);     // n_f strengths
    float2* A = pa + a.n_f + (a.n_f & 1);                   // n_fine
    float2* B = A + a.n_fine;                               // n_fine
    __shared__ int s_first;

    const int c = blockIdx.x / a.n_z;
    const int kap = blockIdx.x - c * a.n_z;
    const int tid = threadIdx.x;
    if (tid == 0) s_first = a.n_f;
    const double lmid = llo[c] + (a.n_l / 2) * a.du;
    const double cell = a.du * a.n_fine * (0.5 / kPi);
    __syncthreads();
    for (int f = tid; f < a.n_f; f += blockDim.x) {
        const double kpf = kp[static_cast<size_t>(kap) * a.n_f + f];
        const float w = wk[static_cast<size_t>(kap) * a.n_f + f];
        const float2 s = spec[(static_cast<size_t>(c) * a.n_z + kap) * a.n_f + f];
        pa[f] = cscale(cmul(s, cis(kpf * lmid)), w);
        py[f] = kpf * cell;
        if (w != 0.0f) atomicMin(&s_first, f);
    }
    for (int i = tid; i < a.n_fine; i += blockDim.x) A[i] = make_float2(0.f, 0.f);
    __syncthreads();
    const int f0 = s_first;
    float2* qo = q + (static_cast<size_t>(c) * a.n_z + kap) * a.n_l;
    if (f0 >= a.n_f) {  // nothing propagates at this k_z
        for (int i = tid; i < a.n_l; i += blockDim.x) qo[i] = make_float2(0.f, 0.f);
        return;
    }
    const int klo = static_cast<int>(floor(py[f0] - a.h)) + 1;
    const int khi = static_cast<int>(floor(py[a.n_f - 1] + a.h));
    const int ncell = min(khi - klo + 1, a.n_fine);
    for (int ci = tid; ci < ncell; ci += blockDim.x) {
        const int k = klo + ci;
        const double left = k - a.h;
        int lo = f0, hi = a.n_f;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (py[mid] > left) hi = mid;
            else lo = mid + 1;
        }
        float2 acc = make_float2(0.f, 0.f);
        for (int f = lo; f < a.n_f; ++f) {
            const double d = k - py[f];
            if (d <= -a.h) break;
            const float z = static_cast<float>(d * a.inv_h);
            const float phi = __expf(static_cast<float>(a.beta) * (sqrtf(fmaxf(1.f - z * z, 0.f)) - 1.f));
            acc.x += pa[f].x * phi;
            acc.y += pa[f].y * phi;
        }
        int kk = k % a.n_fine;
        if (kk < 0) kk += a.n_fine;
        A[kk] = acc;
    }
    __syncthreads();
    const float2* res = lds_fft(A, B, a.n_fine, a.n_fine, 1, a.rad, tw, +1, tid, blockDim.x);
    for (int i = tid; i < a.n_l; i += blockDim.x) {
        int m = i - a.n_l / 2;
        if (m < 0) m += a.n_fine;
        qo[i] = cscale(res[m], deap[i]);
    }
}

}  // namespace

size_t nufft_smem_bytes(const HybridPlan& p) {
    return static_cast<size_t>(p.n_f) * 8 + static_cast<size_t>(p.n_f + (p.n_f & 1)) * 8 +
           2ull * p.n_fine * 8;
}

int launch_range_compress_fp32(const HybridPlan& p, const float2* spec, char* ws, float2* q, hipStream_t s) {
    NufftArgs a{};
    a.n_ch = p.n_ch;
    a.n_z = p.n_z;
    a.n_f = p.n_f;
    a.n_l = p.n_l;
    a.n_fine = p.n_fine;
    a.du = p.du;
    a.h = p.h;
    a.inv_h = 1.0 / p.h;
    a.beta = p.beta;
    a.rad = p.fine_rad;
    const size_t smem = nufft_smem_bytes(p);
    if (smem > 65536) return fail(PL_EUNSUPPORTED, "range compression needs %zu bytes of LDS", smem);
    const long long blocks = static_cast<long long>(p.n_ch) * p.n_z;
    if (blocks > 0x7fffffffLL) return fail(PL_EUNSUPPORTED, "too many (channel, k_z) pairs");
    hipLaunchKernelGGL(nufft_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), smem, s, spec,
                       reinterpret_cast<const double*>(ws + p.off_llo), reinterpret_cast<const double*>(ws + p.off_kp),
                       reinterpret_cast<const float*>(ws + p.off_wk), reinterpret_cast<const float2*>(ws + p.off_tw_fine),
                       reinterpret_cast<const float*>(ws + p.off_deap), a, q);
    return check_launch("range compression");
}

}  // namespace pl
