// Range compression, eq. (8a) / (19a), in FP32.  As a type-1 NUFFT: the k'
// samples of one (channel, k_z) pair are spread onto a 2x fine grid with the
// exponential-of-semicircle kernel, transformed by an inverse FFT in LDS and
// deapodised onto the uniform range grid.  Or, without NUFFT, by resampling
// onto a uniform wavenumber grid and the same inverse FFT.
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
            const float phi = __expf(static_cast<float>(a.beta) * (__builtin_amdgcn_sqrtf(fmaxf(1.f - z * z, 0.f)) - 1.f));
            acc.x += pa[f].x * phi;
            acc.y += pa[f].y * phi;
        }
        // the points lie within half the fine grid of cell 0 (|k' du| <= pi / sigma),
        // so every cell index is within one period of [0, n_fine)
        A[k < 0 ? k + a.n_fine : (k >= a.n_fine ? k - a.n_fine : k)] = acc;
    }
    __syncthreads();
    const float2* res = lds_fft(A, B, a.n_fine, a.n_fine, 1, a.rad, tw, +1, tid, blockDim.x);
    for (int i = tid; i < a.n_l; i += blockDim.x) {
        int m = i - a.n_l / 2;
        if (m < 0) m += a.n_fine;
        qo[i] = cscale(res[m], deap[i]);
    }
}

struct ResampleArgs {
    int n_ch, n_z, n_f, n_l, n_fine, block, bspline;
    int pad_;
    double du, dkl, k0, inv_dk, scan_step;
    double kref[kMaxBlocks];
    Radices rad;
};

// Range compression without NUFFT: resampling onto a uniform k_L grid and an
// inverse FFT.  One block per (channel c, k_z bin kap).  With k_L the
// wavenumber of the path length L = rho_T + rho_R, k_L dk_L = k dk turns the
// frequency sum into (dkl / dk) sum_m k_L,m S(k_m) exp(j k_L,m L) over the
// grid k_L,m = m dkl, k_m = sqrt(k_L,m^2 + k_z^2 / 4).  S(k_m) is a centred
// 4-point Lagrange interpolation over the frequency index of the spectrum
// demodulated by exp(+j k' L_ref), remodulated by exp(-j k' L_ref).
// The planner puts every k_ref on the grid (k_ref = m0 dkl), so
// k'_m = k_L,m - k_ref = n dkl with n = m - m0; with l_i = l_mid + (i - n_l/2) du
// and dkl du = 2 pi / n_fine,
//   q[i] = IFFT(A)[(i - n_l/2) mod n_fine],
//   A[n mod n_fine] = S(k_m) k_L,m (dkl / dk) pf(k'_m) exp(j k'_m (l_mid - L_ref)),
// pf the B-spline prefilter of the back-projection's interpolation.  A block's
// band holds fewer than n_fine grid points (checked by the planner), so no two
// share a bin, and |n| <= n_fine / 2.
__global__ __launch_bounds__(256) void resample_kernel(const float2* __restrict__ spec,
                                                      const double* __restrict__ llo,
                                                      const double* __restrict__ lref,
                                                      const double* __restrict__ kp,
                                                      const float* __restrict__ wk,
                                                      const float2* __restrict__ tw, ResampleArgs a,
                                                      float2* __restrict__ q) {
    extern __shared__ double smem_d[];
    float2* pa = reinterpret_cast<float2*>(smem_d);         // n_f demodulated samples
    float2* A = pa + a.n_f + (a.n_f & 1);                   // n_fine
    float2* B = A + a.n_fine;                               // n_fine
    __shared__ int s_first;

    const int c = blockIdx.x / a.n_z;
    const int kap = blockIdx.x - c * a.n_z;
    const int tid = threadIdx.x;
    if (tid == 0) s_first = a.n_f;
    const double lmid = llo[c] + (a.n_l / 2) * a.du;
    const double lr = lref[c];
    const double kr0 = a.kref[kap / a.block];
    const double* kprow = kp + static_cast<size_t>(kap) * a.n_f;
    __syncthreads();
    for (int f = tid; f < a.n_f; f += blockDim.x) {
        const float2 s = spec[(static_cast<size_t>(c) * a.n_z + kap) * a.n_f + f];
        pa[f] = cmul(s, cis(kprow[f] * lr));
        if (wk[static_cast<size_t>(kap) * a.n_f + f] != 0.0f) atomicMin(&s_first, f);
    }
    for (int i = tid; i < a.n_fine; i += blockDim.x) A[i] = make_float2(0.f, 0.f);
    __syncthreads();
    const int f0 = s_first;
    float2* qo = q + (static_cast<size_t>(c) * a.n_z + kap) * a.n_l;
    if (f0 >= a.n_f) {  // nothing propagates at this k_z
        for (int i = tid; i < a.n_l; i += blockDim.x) qo[i] = make_float2(0.f, 0.f);
        return;
    }
    const int sk = kap < (a.n_z + 1) / 2 ? kap : kap - a.n_z;
    const double kz = 2.0 * kPi * sk / (a.n_z * a.scan_step);
    const double kz2q = 0.25 * kz * kz;
    const long long m_lo = static_cast<long long>(ceil((kprow[f0] + kr0) / a.dkl - 1e-9));
    const long long m_hi = static_cast<long long>(floor((kprow[a.n_f - 1] + kr0) / a.dkl + 1e-9));
    const long long m0 = llround(kr0 / a.dkl);
    const int n_pts = min(4, a.n_f - f0);
    const double dl = lmid - lr;
    const float wscale = static_cast<float>(a.dkl * a.inv_dk);
    for (long long m = m_lo + tid; m <= m_hi; m += blockDim.x) {
        const double kl = static_cast<double>(m) * a.dkl;
        const double t = (sqrt(kl * kl + kz2q) - a.k0) * a.inv_dk;
        const int st = min(max(static_cast<int>(floor(t)) - 1, f0), a.n_f - n_pts);
        const float x = static_cast<float>(t - st);   // nodes at 0 .. n_pts-1
        float w[4];
        if (n_pts == 4) {
            const float a0 = x, a1 = x - 1.f, a2 = x - 2.f, a3 = x - 3.f;
            w[0] = -(1.f / 6.f) * a1 * a2 * a3;
            w[1] = 0.5f * a0 * a2 * a3;
            w[2] = -0.5f * a0 * a1 * a3;
            w[3] = (1.f / 6.f) * a0 * a1 * a2;
        } else {  // 1-3 propagating samples: all of them
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float wj = j < n_pts ? 1.f : 0.f;
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    if (i != j && i < n_pts) wj *= (x - i) / static_cast<float>(j - i);
                w[j] = wj;
            }
        }
        float2 v = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float2 pj = pa[min(st + j, a.n_f - 1)];
            v.x += w[j] * pj.x;
            v.y += w[j] * pj.y;
        }
        const int n = static_cast<int>(m - m0);
        const double kpm = n * a.dkl;
        float scale = static_cast<float>(kl) * wscale;
        if (a.bspline) {
            // |k' du / 2| <= pi / (2 sigma) + pi / n_fine < 0.8: the Taylor
            // series of sin(y)/y to y^10 is exact to 1e-11 there
            const float y = static_cast<float>(0.5 * kpm * a.du), y2 = y * y;
            const float sinc =
                1.f + y2 * (-1.f / 6 + y2 * (1.f / 120 + y2 * (-1.f / 5040 + y2 * (1.f / 362880 - y2 * (1.f / 39916800)))));
            scale /= (sinc * sinc) * (sinc * sinc);
        }
        A[n < 0 ? n + a.n_fine : n] = cscale(cmul(v, cis(kpm * dl)), scale);
    }
    __syncthreads();
    const float2* res = lds_fft(A, B, a.n_fine, a.n_fine, 1, a.rad, tw, +1, tid, blockDim.x);
    for (int i = tid; i < a.n_l; i += blockDim.x) {
        int mm = i - a.n_l / 2;
        if (mm < 0) mm += a.n_fine;
        qo[i] = res[mm];
    }
}

// ---------------------------------------------------------------------------
// Wavefront-per-pair form for fine grids of N = 64 R points (R 2,3,5-smooth,
// at most 32): one wavefront owns one (channel, k_z) pair and its LDS, so
// the kernel has no workgroup barriers; the inverse FFT is wave_ifft.

struct NufftWaveArgs {
    int n_z, n_f, n_l, n_pairs;
    double du, h, beta, inv_h;
};

// LDS of one wavefront: n_f positions (double), n_f strengths, R rows.
constexpr size_t nufft_wave_lds(int r, int n_f) { return 16ull * n_f + 8ull * r * kWaveRow; }

// One workgroup (one wavefront) per (channel c, k_z bin kap); the same
// strengths, spreading and deapodisation as nufft_kernel.
template <int R>
__global__ __launch_bounds__(64) void nufft_wave_kernel(const float2* __restrict__ spec,
                                                       const double* __restrict__ llo,
                                                       const double* __restrict__ kp,
                                                       const float* __restrict__ wk,
                                                       const float2* __restrict__ tw,
                                                       const float* __restrict__ deap, NufftWaveArgs a,
                                                       float2* __restrict__ q) {
    constexpr int N = 64 * R;
    extern __shared__ double smem_d[];
    double* py = smem_d;                                  // n_f fine-grid positions
    float2* pa = reinterpret_cast<float2*>(py + a.n_f);   // n_f strengths
    float2* A = pa + a.n_f;                               // R rows of kWaveRow
    const int lane = threadIdx.x;
    const int pair = blockIdx.x;                          // = c * n_z + kap
    const int c = pair / a.n_z;
    const int kap = pair - c * a.n_z;
    const double lmid = llo[c] + (a.n_l / 2) * a.du;
    const double cell = a.du * N * (0.5 / kPi);

    // strengths and positions; first propagating frequency by ballot
    int f0 = a.n_f;
    for (int fb = 0; fb < a.n_f; fb += 64) {
        const int f = fb + lane;
        float w = 0.f;
        if (f < a.n_f) {
            const double kpf = kp[static_cast<size_t>(kap) * a.n_f + f];
            w = wk[static_cast<size_t>(kap) * a.n_f + f];
            const float2 sv = spec[static_cast<size_t>(pair) * a.n_f + f];
            pa[f] = cscale(cmul(sv, cis(kpf * lmid)), w);
            py[f] = kpf * cell;
        }
        const unsigned long long m = __ballot(w != 0.0f);
        if (f0 == a.n_f && m) f0 = fb + __ffsll(static_cast<long long>(m)) - 1;
    }
    float2* qo = q + static_cast<size_t>(pair) * a.n_l;
    if (f0 >= a.n_f) {  // nothing propagates at this k_z
        for (int i = lane; i < a.n_l; i += 64) qo[i] = make_float2(0.f, 0.f);
        return;
    }
#pragma unroll
    for (int j = 0; j < R; ++j) A[64 * j + lane] = make_float2(0.f, 0.f);
    wave_lds_sync();

    // spreading onto the fine grid: each cell gathers its neighbours (the
    // positions rise with f) found by binary search
    const int klo = static_cast<int>(floor(py[f0] - a.h)) + 1;
    const int khi = static_cast<int>(floor(py[a.n_f - 1] + a.h));
    const int ncell = min(khi - klo + 1, N);
    for (int ci = lane; ci < ncell; ci += 64) {
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
            const float phi = __expf(static_cast<float>(a.beta) * (__builtin_amdgcn_sqrtf(fmaxf(1.f - z * z, 0.f)) - 1.f));
            acc.x += pa[f].x * phi;
            acc.y += pa[f].y * phi;
        }
        // every cell index is within one period of [0, N) (see nufft_kernel)
        A[k < 0 ? k + N : (k >= N ? k - N : k)] = acc;
    }
    wave_lds_sync();

    const int half = a.n_l / 2;
    const float* dp = deap;
    wave_ifft<R>(A, tw, lane, [&](int k, float2 v) {
        // deapodised into q[i] for k = (i - n_l / 2) mod N
        const int i = k < half ? k + half : k - N + half;
        if (i >= 0 && i < a.n_l) qo[i] = cscale(v, dp[i]);
    });
}

template <int R>
int launch_nufft_wave(const HybridPlan& p, const float2* spec, char* ws, float2* q, hipStream_t s) {
    NufftWaveArgs a{};
    a.n_z = p.n_z;
    a.n_f = p.n_f;
    a.n_l = p.n_l;
    const long long pairs = static_cast<long long>(p.n_ch) * p.n_z;
    if (pairs > 0x7fffffffLL) return fail(PL_EUNSUPPORTED, "too many (channel, k_z) pairs");
    a.n_pairs = static_cast<int>(pairs);
    a.du = p.du;
    a.h = p.h;
    a.inv_h = 1.0 / p.h;
    a.beta = p.beta;
    const size_t smem = nufft_wave_lds(R, p.n_f);
    auto fn = nufft_wave_kernel<R>;
    if (smem > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem));
        if (e != hipSuccess) return fail(PL_EDEVICE, "range compression LDS of %zu bytes: %s", smem, hipGetErrorString(e));
    }
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(pairs)), dim3(64), smem, s, spec,
                       reinterpret_cast<const double*>(ws + p.off_llo), reinterpret_cast<const double*>(ws + p.off_kp),
                       reinterpret_cast<const float*>(ws + p.off_wk), reinterpret_cast<const float2*>(ws + p.off_tw_fine),
                       reinterpret_cast<const float*>(ws + p.off_deap), a, q);
    return check_launch("range compression (wavefront per pair)");
}

// Wavefront-per-pair form of resample_kernel for fine grids of N = 64 R
// points (the same uniform-grid samples; the FFT of nufft_wave_kernel).
template <int R>
__global__ __launch_bounds__(64) void resample_wave_kernel(const float2* __restrict__ spec,
                                                          const double* __restrict__ llo,
                                                          const double* __restrict__ lref,
                                                          const double* __restrict__ kp,
                                                          const float* __restrict__ wk,
                                                          const float2* __restrict__ tw, ResampleArgs a,
                                                          float2* __restrict__ q) {
    constexpr int N = 64 * R;
    extern __shared__ double smem_d[];
    float2* pa = reinterpret_cast<float2*>(smem_d);   // n_f demodulated samples
    float2* A = pa + a.n_f;                           // R rows of kWaveRow
    const int lane = threadIdx.x;
    const int pair = blockIdx.x;                      // = c * n_z + kap
    const int c = pair / a.n_z;
    const int kap = pair - c * a.n_z;
    const double lmid = llo[c] + (a.n_l / 2) * a.du;
    const double lr = lref[c];
    const double kr0 = a.kref[kap / a.block];
    const double* kprow = kp + static_cast<size_t>(kap) * a.n_f;

    int f0 = a.n_f;
    for (int fb = 0; fb < a.n_f; fb += 64) {
        const int f = fb + lane;
        float w = 0.f;
        if (f < a.n_f) {
            const float2 sv = spec[static_cast<size_t>(pair) * a.n_f + f];
            pa[f] = cmul(sv, cis(kprow[f] * lr));
            w = wk[static_cast<size_t>(kap) * a.n_f + f];
        }
        const unsigned long long m = __ballot(w != 0.0f);
        if (f0 == a.n_f && m) f0 = fb + __ffsll(static_cast<long long>(m)) - 1;
    }
    float2* qo = q + static_cast<size_t>(pair) * a.n_l;
    if (f0 >= a.n_f) {  // nothing propagates at this k_z
        for (int i = lane; i < a.n_l; i += 64) qo[i] = make_float2(0.f, 0.f);
        return;
    }
#pragma unroll
    for (int j = 0; j < R; ++j) A[64 * j + lane] = make_float2(0.f, 0.f);
    wave_lds_sync();

    const int sk = kap < (a.n_z + 1) / 2 ? kap : kap - a.n_z;
    const double kz = 2.0 * kPi * sk / (a.n_z * a.scan_step);
    const double kz2q = 0.25 * kz * kz;
    const long long m_lo = static_cast<long long>(ceil((kprow[f0] + kr0) / a.dkl - 1e-9));
    const long long m_hi = static_cast<long long>(floor((kprow[a.n_f - 1] + kr0) / a.dkl + 1e-9));
    const long long m0 = llround(kr0 / a.dkl);
    const int n_pts = min(4, a.n_f - f0);
    const double dl = lmid - lr;
    const float wscale = static_cast<float>(a.dkl * a.inv_dk);
    for (long long m = m_lo + lane; m <= m_hi; m += 64) {
        const double kl = static_cast<double>(m) * a.dkl;
        const double t = (sqrt(kl * kl + kz2q) - a.k0) * a.inv_dk;
        const int st = min(max(static_cast<int>(floor(t)) - 1, f0), a.n_f - n_pts);
        const float x = static_cast<float>(t - st);   // nodes at 0 .. n_pts-1
        float w[4];
        if (n_pts == 4) {
            const float a0 = x, a1 = x - 1.f, a2 = x - 2.f, a3 = x - 3.f;
            w[0] = -(1.f / 6.f) * a1 * a2 * a3;
            w[1] = 0.5f * a0 * a2 * a3;
            w[2] = -0.5f * a0 * a1 * a3;
            w[3] = (1.f / 6.f) * a0 * a1 * a2;
        } else {  // 1-3 propagating samples: all of them
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float wj = j < n_pts ? 1.f : 0.f;
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    if (i != j && i < n_pts) wj *= (x - i) / static_cast<float>(j - i);
                w[j] = wj;
            }
        }
        float2 v = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float2 pj = pa[min(st + j, a.n_f - 1)];
            v.x += w[j] * pj.x;
            v.y += w[j] * pj.y;
        }
        const int n = static_cast<int>(m - m0);
        const double kpm = n * a.dkl;
        float scale = static_cast<float>(kl) * wscale;
        if (a.bspline) {
            const float y = static_cast<float>(0.5 * kpm * a.du), y2 = y * y;
            const float sinc =
                1.f + y2 * (-1.f / 6 + y2 * (1.f / 120 + y2 * (-1.f / 5040 + y2 * (1.f / 362880 - y2 * (1.f / 39916800)))));
            scale /= (sinc * sinc) * (sinc * sinc);
        }
        A[n < 0 ? n + N : n] = cscale(cmul(v, cis(kpm * dl)), scale);
    }
    wave_lds_sync();

    const int half = a.n_l / 2;
    wave_ifft<R>(A, tw, lane, [&](int k, float2 v) {
        const int i = k < half ? k + half : k - N + half;
        if (i >= 0 && i < a.n_l) qo[i] = v;
    });
}

// Fine-grid sizes with a wavefront-per-pair kernel: N = 64 R.
#define PL_NUFFT_WAVE_SIZES(X) \
    X(2) X(3) X(4) X(5) X(6) X(8) X(9) X(10) X(12) X(15) X(16) X(18) X(20) X(24) X(25) X(27) X(30) X(32)

}  // namespace

size_t nufft_smem_bytes(const HybridPlan& p) {
    return static_cast<size_t>(p.n_f) * 8 + static_cast<size_t>(p.n_f + (p.n_f & 1)) * 8 +
           2ull * p.n_fine * 8;
}

int launch_range_compress_fp32(const HybridPlan& p, const float2* spec, char* ws, float2* q, hipStream_t s) {
    if (p.range_method == PL_RANGE_RESAMPLE) return launch_range_compress_resample(p, spec, ws, q, s);
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
    if (p.n_fine % 64 == 0) {
#define PL_NW(R) \
        if (p.n_fine == 64 * R) return launch_nufft_wave<R>(p, spec, ws, q, s);
        PL_NUFFT_WAVE_SIZES(PL_NW)
#undef PL_NW
    }
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

namespace pl {

int launch_range_compress_resample(const HybridPlan& p, const float2* spec, char* ws, float2* q, hipStream_t s) {
    if (p.range_method != PL_RANGE_RESAMPLE || !(p.dkl > 0) || !(p.dk > 0))
        return fail(PL_EINVAL, "resampling range compression: plan has no uniform grid");
    ResampleArgs a{};
    a.n_ch = p.n_ch;
    a.n_z = p.n_z;
    a.n_f = p.n_f;
    a.n_l = p.n_l;
    a.n_fine = p.n_fine;
    a.block = p.block;
    a.bspline = p.interp == PL_INTERP_BSPLINE4;
    a.du = p.du;
    a.dkl = p.dkl;
    a.k0 = p.k0;
    a.inv_dk = 1.0 / p.dk;
    a.scan_step = p.scan_step;
    for (int b = 0; b < kMaxBlocks; ++b) a.kref[b] = p.kref[b];
    for (int b = 0; b < p.n_blocks; ++b)
        if (std::fabs(p.kref[b] / p.dkl - std::nearbyint(p.kref[b] / p.dkl)) > 1e-6)
            return fail(PL_EINVAL, "resampling range compression: reference wavenumber off the grid");
    a.rad = p.fine_rad;
    const long long blocks = static_cast<long long>(p.n_ch) * p.n_z;
    if (blocks > 0x7fffffffLL) return fail(PL_EUNSUPPORTED, "too many (channel, k_z) pairs");
    if (p.n_fine % 64 == 0) {
#define PL_RW(R)                                                                                                  \
        if (p.n_fine == 64 * R) {                                                                                 \
            const size_t smem_w = 8ull * p.n_f + 8ull * R * kWaveRow;                                             \
            if (smem_w > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(resample_wave_kernel<R>),    \
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,                 \
                                                      static_cast<int>(smem_w)) != hipSuccess)                    \
                return fail(PL_EDEVICE, "resampling range compression: LDS of %zu bytes refused", smem_w);        \
            hipLaunchKernelGGL(resample_wave_kernel<R>, dim3(static_cast<unsigned>(blocks)), dim3(64), smem_w, s,  \
                               spec, reinterpret_cast<const double*>(ws + p.off_llo),                             \
                               reinterpret_cast<const double*>(ws + p.off_lref),                                  \
                               reinterpret_cast<const double*>(ws + p.off_kp),                                    \
                               reinterpret_cast<const float*>(ws + p.off_wk),                                     \
                               reinterpret_cast<const float2*>(ws + p.off_tw_fine), a, q);                        \
            return check_launch("range compression (resampling, wavefront per pair)");                           \
        }
        PL_NUFFT_WAVE_SIZES(PL_RW)
#undef PL_RW
    }
    const size_t smem = static_cast<size_t>(p.n_f + (p.n_f & 1)) * 8 + 2ull * p.n_fine * 8;
    if (smem > 65536) return fail(PL_EUNSUPPORTED, "resampling range compression needs %zu bytes of LDS", smem);
    hipLaunchKernelGGL(resample_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), smem, s, spec,
                       reinterpret_cast<const double*>(ws + p.off_llo), reinterpret_cast<const double*>(ws + p.off_lref),
                       reinterpret_cast<const double*>(ws + p.off_kp), reinterpret_cast<const float*>(ws + p.off_wk),
                       reinterpret_cast<const float2*>(ws + p.off_tw_fine), a, q);
    return check_launch("range compression (resampling)");
}

}  // namespace pl
